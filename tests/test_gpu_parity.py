"""GPU parity: every libpir entry point against the CPU oracle, bit-exact.

All integer arithmetic mod q, so the bar is exact equality.  Shapes span
several tiles with ragged tails (R not a multiple of 64, C not a multiple
of 8, 2B not a multiple of 8), plus the degenerate R = C = 1 and the largest
batch.
"""

import numpy as np
import pytest

import synth
from oracle import scan as osc
from oracle import query as oq

from pirtest import (empty_dev, expected_columns, freivalds_ok, onehot_queries, residues, ring,
                     sample_columns, to_dev, to_host)

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


@pytest.mark.parametrize("log2n,K", [(10, 1), (10, 2), (11, 2), (12, 2), (12, 1)])
def test_ntt_intt_match_oracle(ctx, log2n, K):
    rg = ring(log2n, K)
    rng = np.random.default_rng(log2n * 10 + K)
    x = residues(rng, (7,), rg)                                 # [7][K][N]
    d = to_dev(x)
    ctx.ntt(rg.pir_params(), d)
    got = to_host(d)
    assert np.array_equal(got, osc.query_ntt(x, rg.primes, rg.psis))
    ctx.intt(rg.pir_params(), d)
    assert np.array_equal(to_host(d), x)


@pytest.mark.parametrize("log2n,K,R,C", [(10, 2, 70, 13), (11, 1, 64, 8), (12, 2, 5, 3),
                                         (10, 1, 1, 1), (11, 2, 33, 17)])
def test_db_load_matches_oracle(ctx, log2n, K, R, C):
    rg = ring(log2n, K)
    raw = synth.db_bytes(R * 100 + C, R, C, rg.N)
    db = ctx.load_db(rg.pir_params(), raw, R, C)
    got = to_host(db.read_ntt(0, R, 0, C))                       # [R][C][K][N]
    exp = osc.db_ntt(raw, rg.primes, rg.psis)                    # [K][R][C][N]
    assert np.array_equal(got, exp.transpose(1, 2, 0, 3))
    db.free()


def test_db_load_from_device_buffer(ctx):
    import torch
    rg = ring(10, 2)
    R, C = 40, 9
    raw = synth.db_bytes(77, R, C, rg.N)
    db = ctx.load_db(rg.pir_params(), torch.from_numpy(raw).to("cuda"), R, C)
    got = to_host(db.read_ntt(3, 30, 2, 5))
    exp = osc.db_ntt(raw[3:33, 2:7], rg.primes, rg.psis)
    assert np.array_equal(got, exp.transpose(1, 2, 0, 3))


SCAN_CASES = [
    # log2n, K, R, C, B
    (10, 2, 100, 21, 1),
    (10, 1, 130, 300, 1),     # two column chunks of the batch-1 kernel
    (11, 2, 64, 8, 1),
    (10, 1, 1, 1, 1),
    (10, 2, 100, 21, 2),
    (10, 2, 100, 21, 3),
    (10, 1, 96, 40, 4),
    (11, 2, 70, 13, 5),
    (10, 2, 129, 35, 17),
    (10, 1, 65, 19, 33),      # two column tiles, ragged
    (10, 1, 3, 2, 256),       # largest batch
    (12, 2, 40, 9, 8),
]


@pytest.mark.parametrize("log2n,K,R,C,B", SCAN_CASES)
def test_db_mul_matches_oracle(ctx, log2n, K, R, C, B):
    rg = ring(log2n, K)
    raw = synth.db_bytes(R + C + B, R, C, rg.N)
    rng = np.random.default_rng(R * C * B)
    q_hat = residues(rng, (B, R, 2), rg)                          # [B][R][2][K][N]
    db = ctx.load_db(rg.pir_params(), raw, R, C)
    out = empty_dev((B, C, 2, K, rg.N))
    ctx.db_mul(db, to_dev(q_hat), B, out)
    got = to_host(out)
    exp = osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis), q_hat, rg.primes)
    assert np.array_equal(got, exp)
    db.free()


def test_db_mul_extreme_residues(ctx):
    """All-(q-1) query and all-255 database: the largest limb sums the kernels meet."""
    rg = ring(10, 2)
    R, C, B = 200, 16, 3
    raw = np.full((R, C, rg.N), 255, dtype=np.uint8)
    q_hat = np.stack([np.full((B, R, 2, rg.N), q - 1, dtype=np.uint64) for q in rg.primes], axis=3)
    db = ctx.load_db(rg.pir_params(), raw, R, C)
    for b in (1, B):
        out = empty_dev((b, C, 2, rg.K, rg.N))
        ctx.db_mul(db, to_dev(q_hat[:b]), b, out)
        exp = osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis), q_hat[:b], rg.primes)
        assert np.array_equal(to_host(out), exp)


def test_small_primes(ctx):
    """Two small primes (12289, 40961: residues of two 7-bit limbs, the upper
    limb planes all zero) with mostly all-255 bytes and all-(q-1) queries;
    every batch-1 and batched variant."""
    from paper_2606_11536_amd import pir
    from pirtest import Ring
    from oracle import params as op
    log2n, R, C = 10, 1000, 10
    N = 1 << log2n
    qs = [12289, 40961]
    rg = Ring(log2n, qs, [op.psi_min(N, q) for q in qs], op.scale(qs, 256))
    raw = np.full((R, C, N), 255, dtype=np.uint8)
    raw[:, :, ::7] = synth.db_bytes(41, R, C, N)[:, :, ::7]
    db = ctx.load_db(rg.pir_params(), raw, R, C)
    dbn = osc.db_ntt(raw, rg.primes, rg.psis)
    for B in (1, 3):
        q_hat = np.stack([np.full((B, R, 2, N), q - 1, dtype=np.uint64) for q in qs], axis=3)
        q_hat[..., ::5] = residues(np.random.default_rng(B), (B, R, 2), rg)[..., ::5]
        exp = osc.db_mul(dbn, q_hat, rg.primes)
        qd = to_dev(q_hat)
        for v in range(pir.scan_variants(B)):
            ctx.scan_select(db, B, v)
            out = empty_dev((B, C, 2, rg.K, N))
            ctx.db_mul(db, qd, B, out)
            assert np.array_equal(to_host(out), exp), f"B={B} variant {v}"
    db.free()


@pytest.mark.parametrize("seed", [0, 5, 15])
def test_tiny_workload_end_to_end(ctx, seed):
    """N=1024, one prime, 16 x 16 DB, one query: GPU answer == oracle; decrypts to row seed % 16."""
    rg = ring(10, 1)
    R = C = 16
    raw = synth.db_bytes(seed, R, C, rg.N)
    i_star = seed % 16
    ct, s = oq.onehot_query(seed, 0, i_star, R, rg.primes, rg.psis, rg.delta, rg.N)
    db = ctx.load_db(rg.pir_params(), raw, R, C)
    qd = to_dev(ct[None])
    out = empty_dev((1, C, 2, 1, rg.N))
    ctx.answer_batch([(db, 1, qd, out)])
    got = to_host(out)[0]
    y = osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis), osc.query_ntt(ct[None], rg.primes, rg.psis),
                   rg.primes)
    assert np.array_equal(got, osc.answer_intt(y, rg.primes, rg.psis)[0])
    m, noise = oq.decrypt_answers(got, s, rg.primes, rg.psis, rg.delta, rg.p)
    assert np.array_equal(m, raw[i_star].astype(np.int64))
    assert np.array_equal(to_host(qd), ct[None])      # query left unchanged


def test_multi_database_batch(ctx):
    """Three databases of different N, R, C and batch sizes in one call."""
    specs = [(12, 2, 40, 20, 3), (11, 2, 75, 23, 1), (11, 2, 16, 70, 6)]
    rng = np.random.default_rng(3)
    jobs, checks = [], []
    for n, (log2n, K, R, C, B) in enumerate(specs):
        rg = ring(log2n, K)
        raw = synth.db_bytes(500 + n, R, C, rg.N)
        qc = residues(rng, (B, R, 2), rg)
        db = ctx.load_db(rg.pir_params(), raw, R, C)
        out = empty_dev((B, C, 2, K, rg.N))
        jobs.append((db, B, to_dev(qc), out))
        checks.append((rg, raw, qc))
    ctx.answer_batch(jobs)
    for (db, B, qd, out), (rg, raw, qc) in zip(jobs, checks):
        y = osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis), osc.query_ntt(qc, rg.primes, rg.psis),
                       rg.primes)
        assert np.array_equal(to_host(out), osc.answer_intt(y, rg.primes, rg.psis))


def test_batch1_full_size(ctx):
    """N=2048, two primes, 512 x 256 DB (256 MiB raw), one encrypted query.

    Checks: 16+ sampled columns exactly, two Freivalds draws per prime over
    the whole answer, and decryption of every column to the selected row --
    for both the NTT-form entry point and the fused coefficient-form batch.
    """
    rg = ring(11, 2)
    R, C, seed = 512, 256, 0
    raw = synth.db_bytes(seed, R, C, rg.N)
    i_star = seed % R
    ct, s = onehot_queries(seed, np.array([i_star]), R, rg)
    q_hat = osc.query_ntt(ct, rg.primes, rg.psis)
    db = ctx.load_db(rg.pir_params(), raw, R, C)
    out = empty_dev((1, C, 2, 2, rg.N))
    ctx.db_mul(db, to_dev(q_hat), 1, out)
    ans_ntt = to_host(out)
    cols = sample_columns(C, 16, seed)
    assert np.array_equal(ans_ntt[:, cols], expected_columns(raw, q_hat, cols, rg))
    assert freivalds_ok(raw, q_hat, ans_ntt, rg, seed, coeff_form=False)

    out2 = empty_dev((1, C, 2, 2, rg.N))
    ctx.answer_batch([(db, 1, to_dev(ct), out2)])
    ans = to_host(out2)
    assert np.array_equal(ans, osc.answer_intt(ans_ntt, rg.primes, rg.psis))
    m, noise = oq.decrypt_answers(ans[0], s[0], rg.primes, rg.psis, rg.delta, rg.p)
    assert np.array_equal(m, raw[i_star].astype(np.int64))
    assert max(abs(int(v)) for v in noise.ravel()) < rg.delta // 2


@pytest.mark.parametrize("log2n,K,R,C,B", [(10, 2, 200, 45, 1), (11, 1, 130, 300, 1),
                                           (10, 2, 512, 45, 1), (10, 1, 2560, 20, 1),
                                           (10, 2, 200, 45, 3), (10, 1, 97, 70, 5),
                                           (10, 1, 97, 70, 17), (10, 2, 300, 41, 33),
                                           (10, 1, 64, 33, 64)])
def test_every_scan_variant_matches_oracle(ctx, log2n, K, R, C, B):
    from paper_2606_11536_amd import pir
    rg = ring(log2n, K)
    raw = synth.db_bytes(7 * R + C, R, C, rg.N)
    rng = np.random.default_rng(R + 3 * C + B)
    q_hat = residues(rng, (B, R, 2), rg)
    db = ctx.load_db(rg.pir_params(), raw, R, C)
    exp = osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis), q_hat, rg.primes)
    qd = to_dev(q_hat)
    n = pir.scan_variants(B)
    assert n >= 2
    for v in range(n):
        ctx.scan_select(db, B, v)
        out = empty_dev((B, C, 2, K, rg.N))
        ctx.db_mul(db, qd, B, out)
        assert np.array_equal(to_host(out), exp), f"variant {v}"
    report = ctx.tune(db, B)
    assert "best=" in report
    out = empty_dev((B, C, 2, K, rg.N))
    ctx.db_mul(db, qd, B, out)
    assert np.array_equal(to_host(out), exp)


def test_scan_kernel_names(ctx):
    """The default batch-1 variant runs the ring kernel when every query chunk's
    k-block count is a multiple of its depth (R = 512: 8 k-blocks; R = 200: 4),
    else the grouped kernel (R = 130: 3 k-blocks); B > 1 runs the MFMA kernel."""
    rg = ring(10, 1)
    names = {}
    for R in (512, 200, 130):
        db = ctx.load_db(rg.pir_params(), synth.db_bytes(R, R, 9, rg.N), R, 9)
        names[R] = (ctx.scan_kernel(db, 1), ctx.scan_kernel(db, 3))
        db.free()
    assert names == {512: ("k_scan_b1r", "k_scan_mfma"), 200: ("k_scan_b1r", "k_scan_mfma"),
                     130: ("k_scan_b1", "k_scan_mfma")}


@pytest.mark.parametrize("B", [1, 3])
def test_stage_profiling_masks(ctx, B):
    """Scan-only profiling times every scan launch (events recorded by the
    launch) and no other stage; full profiling times every stage; the answers
    are the oracle's either way."""
    rg = ring(10, 1)
    R, C = 64, 9
    raw = synth.db_bytes(41 + B, R, C, rg.N)
    db = ctx.load_db(rg.pir_params(), raw, R, C)
    qc = residues(np.random.default_rng(B), (B, R, 2), rg)
    exp = osc.answer_intt(osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis),
                                     osc.query_ntt(qc, rg.primes, rg.psis), rg.primes),
                          rg.primes, rg.psis)
    qd = to_dev(qc)
    out = empty_dev((B, C, 2, 1, rg.N))
    ctx.profile(True, stages=("scan",))
    for _ in range(3):
        ctx.answer_batch([(db, B, qd, out)])
    scan, ntt = ctx.profile_read("scan"), ctx.profile_read("ntt")
    assert scan[1] == 3 and scan[0] > 0 and ntt == (0.0, 0)
    ctx.profile(True)
    ctx.answer_batch([(db, B, qd, out)])
    for st in ("ntt", "scan", "intt") + (("pack", "unpack") if B > 1 else ()):
        assert ctx.profile_read(st)[1] == 1, st
    ctx.profile(False)
    assert np.array_equal(to_host(out), exp)
    db.free()


def test_fused_batch_many_jobs_and_tuning(ctx):
    """Eleven jobs over four databases (mixed N, R, C, B, including B = 1): the
    fused scan launches split at eight jobs; every variant choice made by
    pir_tune_batch gives the same bytes."""
    specs = [(10, 2, 90, 19), (11, 2, 64, 33), (12, 2, 20, 12), (10, 1, 130, 9)]
    Bs = [1, 3, 2, 7, 1, 12, 5, 4, 1, 9, 2]
    rng = np.random.default_rng(21)
    dbs = []
    for n, (log2n, K, R, C) in enumerate(specs):
        rg = ring(log2n, K)
        raw = synth.db_bytes(900 + n, R, C, rg.N)
        dbs.append((rg, raw, ctx.load_db(rg.pir_params(), raw, R, C), R, C))
    jobs, checks = [], []
    for n, B in enumerate(Bs):
        rg, raw, db, R, C = dbs[n % len(dbs)]
        qc = residues(rng, (B, R, 2), rg)
        out = empty_dev((B, C, 2, rg.K, rg.N))
        jobs.append((db, B, to_dev(qc), out))
        checks.append((rg, raw, qc))
    exp = []
    for rg, raw, qc in checks:
        y = osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis), osc.query_ntt(qc, rg.primes, rg.psis),
                       rg.primes)
        exp.append(osc.answer_intt(y, rg.primes, rg.psis))
    ctx.answer_batch(jobs)
    for (_, _, _, out), e in zip(jobs, exp):
        assert np.array_equal(to_host(out), e)
    report = ctx.tune_batch(jobs)
    assert "best=" in report
    for (_, _, _, out) in jobs:
        out.zero_()
    ctx.answer_batch(jobs)
    for (_, _, _, out), e in zip(jobs, exp):
        assert np.array_equal(to_host(out), e)
