"""GPU parity of the scalar-HE database GEMM mod 2^32 (pir_sdb_load / pir_sdb_mul).

* word for word against the oracle over ragged shapes (D1 and D0 not
  multiples of the 32 x 32 tiles, one row, one column) and every batch-size
  regime of the kernel (one, two and four column blocks of 8 queries, and
  batches that leave a block partly empty);
* extreme operands: every entry -128 or 127, every word 2^32 - 1 or
  0x80808080 (digits at the ends of their range);
* D0 at its limit (131071) with the largest products, sampled rows;
* a toy SimplePIR round trip: one-hot LWE queries for several columns,
  answered on the GPU, decrypt to the selected database columns;
* a database given in host memory equals the same one given on the device;
* argument checks (D0 past the limit, B = 0).
"""

import numpy as np
import pytest

from oracle import scalar as oscl

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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _run(ctx, db, q):
    import torch
    D1, D0 = db.shape
    B = q.shape[0]
    sdb = ctx.load_sdb(_dev(db), D1, D0)
    out = torch.empty((B, D1), dtype=torch.int32, device="cuda")
    ctx.sdb_mul(sdb, _dev(q.view(np.int32)), B, out)
    got = out.cpu().numpy().view(np.uint32)
    sdb.free()
    return got


@pytest.mark.parametrize("D1,D0,B", [(1, 1, 1), (33, 70, 1), (100, 300, 8), (64, 257, 9),
                                     (97, 1000, 16), (130, 515, 17), (256, 2048, 32),
                                     (40, 100, 45), (70, 90, 256)])
def test_matches_oracle(ctx, D1, D0, B):
    rng = np.random.default_rng(D1 * 1000 + D0 + B)
    db = rng.integers(-128, 128, (D1, D0), dtype=np.int64).astype(np.int8)
    q = rng.integers(0, 1 << 32, (B, D0), dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(_run(ctx, db, q), oscl.db_gemm(db, q))


@pytest.mark.parametrize("entry,word", [(-128, 0xFFFFFFFF), (127, 0x80808080), (-128, 0x80808080),
                                        (127, 0x7F7F7F7F)])
def test_extreme_operands(ctx, entry, word):
    D1, D0, B = 70, 4000, 3
    db = np.full((D1, D0), entry, dtype=np.int8)
    q = np.full((B, D0), word, dtype=np.uint32)
    assert np.array_equal(_run(ctx, db, q), oscl.db_gemm(db, q))


def test_d0_at_the_limit(ctx):
    D1, D0, B = 40, 131071, 2
    rng = np.random.default_rng(17)
    db = np.where(rng.integers(0, 2, (D1, D0)) == 1, -128, 127).astype(np.int8)
    q = np.full((B, D0), 0x80808080, dtype=np.uint32)
    q[1] = rng.integers(0, 1 << 32, D0, dtype=np.uint64).astype(np.uint32)
    got = _run(ctx, db, q)
    rows = [0, 1, 17, D1 - 1]
    assert np.array_equal(got[:, rows], oscl.db_gemm(db[rows], q))


def test_simplepir_round_trip(ctx):
    import torch
    D1, D0, n = 300, 2048, 64
    rng = np.random.default_rng(23)
    db = rng.integers(-128, 128, (D1, D0), dtype=np.int64).astype(np.int8)
    A = rng.integers(0, 1 << 32, (D0, n), dtype=np.uint64).astype(np.uint32)
    s = rng.integers(-1, 2, n, dtype=np.int64)
    sdb = ctx.load_sdb(_dev(db), D1, D0)
    # the hint (D1 x n) is the same GEMM with the columns of A as queries
    hint = torch.empty((n, D1), dtype=torch.int32, device="cuda")
    ctx.sdb_mul(sdb, _dev(A.T.copy().view(np.int32)), n, hint)
    hint = hint.cpu().numpy().view(np.uint32)
    assert np.array_equal(hint, oscl.db_gemm(db, A.T.copy()))
    hint_s = (hint.astype(np.int64).T @ s) % (1 << 32)
    cols = [0, 5, 777, D0 - 1]
    cts = np.stack([oscl.lwe_onehot(A, s, rng.integers(-4, 5, D0, dtype=np.int64), c) for c in cols])
    ans = torch.empty((len(cols), D1), dtype=torch.int32, device="cuda")
    ctx.sdb_mul(sdb, _dev(cts.view(np.int32)), len(cols), ans)
    ans = ans.cpu().numpy().view(np.uint32)
    for n_, c in enumerate(cols):
        assert np.array_equal(oscl.lwe_decrypt(ans[n_], hint_s), db[:, c].astype(np.int64) % 256)
    sdb.free()


def test_host_database(ctx):
    import torch
    D1, D0, B = 77, 333, 5
    rng = np.random.default_rng(5)
    db = rng.integers(-128, 128, (D1, D0), dtype=np.int64).astype(np.int8)
    q = rng.integers(0, 1 << 32, (B, D0), dtype=np.uint64).astype(np.uint32)
    sdb = ctx.load_sdb(db, D1, D0)           # numpy: host memory
    out = torch.empty((B, D1), dtype=torch.int32, device="cuda")
    ctx.sdb_mul(sdb, _dev(q.view(np.int32)), B, out)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), oscl.db_gemm(db, q))
    sdb.free()


def test_arguments(ctx):
    from paper_2606_11536_amd import pir
    with pytest.raises(pir.PirError):
        ctx.load_sdb(np.zeros((2, 131072), dtype=np.int8), 2, 131072)
    sdb = ctx.load_sdb(np.zeros((2, 8), dtype=np.int8), 2, 8)
    q = _dev(np.zeros((1, 8), dtype=np.int32))
    out = _dev(np.zeros((1, 2), dtype=np.int32))
    with pytest.raises(pir.PirError):
        ctx.sdb_mul(sdb, q, 0, out)
    sdb.free()
