"""Pins for oracle.scan and oracle.query.

* the scan in NTT form, drained by the INTT, equals the ring definition
  (schoolbook negacyclic products summed over rows) on tiny inputs;
* trivial query (a = 0, e = 0, b = Delta * one-hot) has the closed form
  answer (0, Delta * NTT(lift(DB[i*][j])));
* identity database returns the query unchanged; the scan is linear in
  the query;
* the tiny workload end to end (N = 1024, one prime, 16 x 16, p = 2^8):
  decryption returns database row i* = seed mod 16 exactly, for seeds 0..15
  (every row), with the noise inside (-Delta/2, Delta/2);
* the Freivalds identity holds on a correct answer and catches a single
  flipped bit planted in it.
"""

import numpy as np
import pytest

import synth
from oracle import ntt, params, query, scan


def _setup(N, K, bound=1 << 28):
    qs = params.ntt_primes(N, K, bound=bound)
    psis = [params.psi_min(N, q) for q in qs]
    return qs, psis


def test_ntt_scan_equals_ring_definition():
    N, R, C, B = 16, 3, 2, 2
    qs, psis = _setup(N, 2, bound=1 << 14)
    rng = np.random.default_rng(5)
    raw = rng.integers(0, 256, size=(R, C, N), dtype=np.uint8)
    qry = np.stack([rng.integers(0, q, size=(B, R, 2, N)) for q in qs], axis=3).astype(np.uint64)
    y = scan.db_mul(scan.db_ntt(raw, qs, psis), scan.query_ntt(qry, qs, psis), qs)
    got = scan.answer_intt(y, qs, psis)
    assert np.array_equal(got, scan.db_mul_coeff(raw, qry, qs))


def test_scan_slot_and_column_selection():
    N, R, C, B = 32, 4, 5, 2
    qs, psis = _setup(N, 2, bound=1 << 16)
    rng = np.random.default_rng(6)
    raw = rng.integers(0, 256, size=(R, C, N), dtype=np.uint8)
    qh = np.stack([rng.integers(0, q, size=(B, R, 2, N)) for q in qs], axis=3).astype(np.uint64)
    dh = scan.db_ntt(raw, qs, psis)
    full = scan.db_mul(dh, qh, qs)
    cols, slots = np.array([0, 3, 4]), np.array([1, 7, 31])
    part = scan.db_mul(dh, qh, qs, slots=slots, cols=cols)
    assert np.array_equal(part, full[:, cols][..., slots])


def test_trivial_query_closed_form():
    N, R, C = 1024, 4, 3
    qs, psis = _setup(N, 1)
    q = qs[0]
    delta = params.scale(qs, 256)
    raw = synth.db_bytes(2, R, C, N)
    i_star = 2
    qry = np.zeros((1, R, 2, 1, N), dtype=np.uint64)
    qry[0, i_star, 1, 0, 0] = delta % q
    y = scan.db_mul(scan.db_ntt(raw, qs, psis), scan.query_ntt(qry, qs, psis), qs)
    assert np.all(y[:, :, 0] == 0)
    for j in range(C):
        expect = ntt.ntt(raw[i_star, j].astype(np.uint64), q, psis[0]) * np.uint64(delta % q) % np.uint64(q)
        assert np.array_equal(y[0, j, 1, 0], expect)


def test_identity_database_returns_query():
    N, R = 64, 4
    qs, psis = _setup(N, 2, bound=1 << 16)
    raw = np.zeros((R, R, N), dtype=np.uint8)
    for i in range(R):
        raw[i, i, 0] = 1
    rng = np.random.default_rng(8)
    qh = np.stack([rng.integers(0, q, size=(1, R, 2, N)) for q in qs], axis=3).astype(np.uint64)
    y = scan.db_mul(scan.db_ntt(raw, qs, psis), qh, qs)
    assert np.array_equal(y, qh)


def test_scan_is_linear_in_query():
    N, R, C = 64, 5, 3
    qs, psis = _setup(N, 2, bound=1 << 16)
    rng = np.random.default_rng(9)
    raw = rng.integers(0, 256, size=(R, C, N), dtype=np.uint8)
    dh = scan.db_ntt(raw, qs, psis)
    q1 = np.stack([rng.integers(0, q, size=(1, R, 2, N)) for q in qs], axis=3).astype(np.uint64)
    q2 = np.stack([rng.integers(0, q, size=(1, R, 2, N)) for q in qs], axis=3).astype(np.uint64)
    qsum = q1.copy()
    for k, q in enumerate(qs):
        qsum[..., k, :] = (q1[..., k, :] + q2[..., k, :]) % np.uint64(q)
    y1, y2, ys = (scan.db_mul(dh, x, qs) for x in (q1, q2, qsum))
    for k, q in enumerate(qs):
        assert np.array_equal(ys[..., k, :], (y1[..., k, :] + y2[..., k, :]) % np.uint64(q))


def tiny_end_to_end(seed):
    """Tiny workload: N = 1024, q = largest prime < 2^28 with q = 1 mod 2N, 16 x 16 DB."""
    N, R, C, p = 1024, 16, 16, 256
    qs, psis = _setup(N, 1)
    delta = params.scale(qs, p)
    raw = synth.db_bytes(seed, R, C, N)
    i_star = seed % 16
    ct, s = query.onehot_query(seed, 0, i_star, R, qs, psis, delta, N)
    y = scan.db_mul(scan.db_ntt(raw, qs, psis), scan.query_ntt(ct[None], qs, psis), qs)
    ans = scan.answer_intt(y, qs, psis)[0]                   # [C][2][K][N]
    m, noise = query.decrypt_answers(ans, s, qs, psis, delta, p)
    return raw, i_star, m, noise, delta


@pytest.mark.parametrize("seed", range(16))
def test_tiny_workload_returns_selected_row(seed):
    raw, i_star, m, noise, delta = tiny_end_to_end(seed)
    assert np.array_equal(m, raw[i_star].astype(np.int64))
    assert max(abs(int(v)) for v in noise.ravel()) < delta // 2


def test_freivalds_identity_and_planted_flip():
    N, R, C, B = 256, 8, 12, 2
    qs, psis = _setup(N, 2)
    raw = synth.db_bytes(4, R, C, N)
    rng = np.random.default_rng(10)
    qh = np.stack([rng.integers(0, q, size=(B, R, 2, N)) for q in qs], axis=3).astype(np.uint64)
    y = scan.db_mul(scan.db_ntt(raw, qs, psis), qh, qs)
    bad = y.copy()
    bad[1, 7, 0, 1, 100] ^= np.uint64(1 << 5)
    for k, (q, psi) in enumerate(zip(qs, psis)):
        for draw in range(2):
            r = synth.freivalds_vector(4, draw, C, q)
            exp = scan.freivalds_expected(raw, qh, r, k, q, psi)
            assert np.array_equal(scan.freivalds_observed(y, r, k, q), exp)
            caught = not np.array_equal(scan.freivalds_observed(bad, r, k, q), exp)
            assert caught == (k == 1)


def test_weighted_rows_multi_brute_force():
    """Several weight vectors and primes in one pass equal sum_j r_j DB[i][j] mod q
    computed with Python integers, including the largest weights q - 1."""
    N, R, C = 8, 5, 37
    qs = params.ntt_primes(16, 2) + [12289]
    raw = synth.db_bytes(8, R, C, N)
    raw[0] = 255
    rng = np.random.default_rng(3)
    rs = [rng.integers(0, q, size=C, dtype=np.uint64) for q in qs]
    rs.append(np.full(C, qs[0] - 1, dtype=np.uint64))
    ps = qs + [qs[0]]
    got = scan.weighted_rows_multi(raw, rs, ps)
    for v, (r, q) in enumerate(zip(rs, ps)):
        for i in range(R):
            for n in range(N):
                exp = sum(int(r[j]) * int(raw[i, j, n]) for j in range(C)) % q
                assert int(got[v, i, n]) == exp
        assert np.array_equal(got[v], scan.weighted_rows(raw, r, q))


def test_freivalds_from_rows_equals_direct():
    N, R, C, B = 64, 6, 9, 3
    qs, psis = _setup(N, 2)
    raw = synth.db_bytes(5, R, C, N)
    rng = np.random.default_rng(11)
    qh = np.stack([rng.integers(0, q, size=(B, R, 2, N)) for q in qs], axis=3).astype(np.uint64)
    y = scan.db_mul(scan.db_ntt(raw, qs, psis), qh, qs)
    rs = [synth.freivalds_vector(5, d, C, q) for q in qs for d in range(2)]
    w = scan.weighted_rows_multi(raw, rs, [q for q in qs for _ in range(2)])
    for v, r in enumerate(rs):
        k = v // 2
        exp = scan.freivalds_expected_from_rows(w[v], qh, k, qs[k], psis[k])
        assert np.array_equal(exp, scan.freivalds_observed(y, r, k, qs[k]))
