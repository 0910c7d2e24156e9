"""Pins for oracle.scalar (Sec. 4.1 INT8-INT32 GEMM mod 2^32; Sec. 2 SimplePIR).

* brute force with Python integers, extreme values included (entries -128
  and 127, words 0 and 2^32 - 1);
* the paper's byte decomposition: four GEMMs over the unsigned bytes of the
  words, shifted by 0, 8, 16, 24 bits and added mod 2^32, give the same
  matrix;
* a toy SimplePIR round trip: a one-hot LWE query for column i*, the
  database GEMM of the query, the hint (the database times the public
  matrix) times the secret, and rounding at scale 2^24 recover column i* of
  the database mod 2^8, for every i* of a small database;
* shape and range checks.
"""

import numpy as np
import pytest

from oracle import scalar as osc

rng = np.random.default_rng(4101)


def _brute(db, q):
    D1, D0 = db.shape
    out = np.zeros((q.shape[0], D1), dtype=np.uint64)
    for b in range(q.shape[0]):
        for r in range(D1):
            out[b, r] = sum(int(db[r, c]) * int(q[b, c]) for c in range(D0)) % (1 << 32)
    return out


@pytest.mark.parametrize("D1,D0,B", [(5, 7, 3), (16, 33, 2), (1, 64, 4)])
def test_brute_force(D1, D0, B):
    db = rng.integers(-128, 128, (D1, D0), dtype=np.int64).astype(np.int8)
    q = rng.integers(0, 1 << 32, (B, D0), dtype=np.uint64).astype(np.uint32)
    db[0, 0], db[-1, -1] = -128, 127
    q[0, 0], q[-1, -1] = (1 << 32) - 1, 0
    assert np.array_equal(osc.db_gemm(db, q).astype(np.uint64), _brute(db, q))


def test_byte_decomposition():
    D1, D0, B = 40, 300, 6
    db = rng.integers(-128, 128, (D1, D0), dtype=np.int64).astype(np.int8)
    q = rng.integers(0, 1 << 32, (B, D0), dtype=np.uint64)
    total = np.zeros((B, D1), dtype=object)
    for k in range(4):
        byte = ((q >> np.uint64(8 * k)) & np.uint64(255)).astype(np.int64)
        part = byte @ db.astype(np.int64).T                 # |part| < 2^8 2^7 300
        total = total + (part.astype(object) << (8 * k))
    want = np.array([[int(v) % (1 << 32) for v in row] for row in total], dtype=np.uint64)
    assert np.array_equal(osc.db_gemm(db, q.astype(np.uint32)).astype(np.uint64), want)


def test_simplepir_round_trip():
    D1, D0, n = 24, 512, 32
    db = rng.integers(-128, 128, (D1, D0), dtype=np.int64).astype(np.int8)
    A = rng.integers(0, 1 << 32, (D0, n), dtype=np.uint64).astype(np.uint32)
    s = rng.integers(-1, 2, n, dtype=np.int64)
    hint = osc.db_gemm(db, A.T.copy())                      # [n][D1] = (DB A)^T mod 2^32
    hint_s = (hint.astype(np.int64).T @ s) % (1 << 32)      # [D1]
    for i_star in range(0, D0, 37):
        e = rng.integers(-4, 5, D0, dtype=np.int64)
        ct = osc.lwe_onehot(A, s, e, i_star)
        ans = osc.db_gemm(db, ct[None])[0]
        got = osc.lwe_decrypt(ans, hint_s)
        assert np.array_equal(got, db[:, i_star].astype(np.int64) % 256)


def test_checks():
    with pytest.raises(ValueError):
        osc.db_gemm(np.zeros((2, 3), dtype=np.uint8), np.zeros((1, 3), dtype=np.uint32))
    with pytest.raises(ValueError):
        osc.db_gemm(np.zeros((2, 3), dtype=np.int8), np.zeros((1, 4), dtype=np.uint32))
