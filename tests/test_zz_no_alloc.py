"""GPU test of pir_answer_batch_static, the entry point that allocates nothing.

It takes the same job lists as pir_answer_batch but keeps its workspace in
the library's fixed device scratch array.  Its answers must equal
pir_answer_batch's word for word:
* first call: a batch-1 job on the 512 x 256 database at N = 2048, two primes
  (16 MiB of NTT-form query in the array), fused with a batched job (B = 3)
  on a ragged database, and a batched switching job (2^29);
* second call, right after, with a smaller job list (N = 1024, one prime,
  B = 3): the array still holds the first call's data;
and a job list whose workspace exceeds the array is refused before anything
runs.  One small case is also checked against the oracle.
"""

import numpy as np
import pytest

import synth
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
    torch.cuda.empty_cache()


def _jobs(ctx, specs, seed):
    """specs: (log2n, K, R, C, B, switch_bits) -> (static jobs, regular jobs, inputs)."""
    rng = np.random.default_rng(seed)
    js, jr, meta = [], [], []
    for n, (log2n, K, R, C, B, bits) in enumerate(specs):
        rg = ring(log2n, K)
        raw = synth.db_bytes(seed + n, R, C, rg.N)
        db = ctx.load_db(rg.pir_params(), raw, R, C)
        qc = residues(rng, (B, R, 2), rg)
        qd = to_dev(qc)
        shape = (B, C, 2, rg.N) if bits else (B, C, 2, K, rg.N)
        js.append((db, B, qd, empty_dev(shape), bits))
        jr.append((db, B, qd, empty_dev(shape), bits))
        meta.append((rg, raw, qc))
    return js, jr, meta


def _run_and_compare(ctx, js, jr):
    import torch
    for (_, _, _, out, _) in js:
        out.fill_(-1)
    ctx.answer_batch_static(js)
    torch.cuda.synchronize()
    ctx.answer_batch(jr)
    torch.cuda.synchronize()
    for n, (s, r) in enumerate(zip(js, jr)):
        assert np.array_equal(to_host(s[3]), to_host(r[3])), f"job {n}"


def test_static_matches_answer_batch_twice(ctx):
    # workspace: 16 MiB of batch-1 query, 4 MiB and 8 MiB of query tiles, ~34 MiB in all
    print("[no-alloc] first call: 512x256 N=2048 B=1, 40x20 N=1024 B=3, 40x20 B=2 switched",
          flush=True)
    js, jr, meta = _jobs(ctx, [(11, 2, 512, 256, 1, 0), (10, 2, 40, 20, 3, 0),
                               (11, 2, 40, 20, 2, 29)], 900)
    _run_and_compare(ctx, js, jr)
    print("[no-alloc] second call: 100x30 N=1024 K=1 B=3", flush=True)
    js2, jr2, meta2 = _jobs(ctx, [(10, 1, 100, 30, 3, 0)], 950)
    _run_and_compare(ctx, js2, jr2)
    rg, raw, qc = meta2[0]
    y = osc.db_mul(osc.db_ntt(raw, rg.primes, rg.psis), osc.query_ntt(qc, rg.primes, rg.psis),
                   rg.primes)
    assert np.array_equal(to_host(js2[0][3]), osc.answer_intt(y, rg.primes, rg.psis))
    for j in js + js2:
        j[0].free()


def test_static_refuses_oversized_job_lists(ctx):
    from paper_2606_11536_amd import pir
    rg = ring(11, 2)
    R, C = 2048, 8                       # one batch-1 query: 2048*2*2*2048*4 = 64 MiB + tail
    db = ctx.load_db(rg.pir_params(), synth.db_bytes(7, R, C, rg.N), R, C)
    import torch
    q = torch.zeros((1, R, 2, 2, rg.N), dtype=torch.int32, device="cuda")
    out = torch.zeros((1, C, 2, 2, rg.N), dtype=torch.int32, device="cuda")
    q2 = torch.zeros((1, 8, 2, 2, rg.N), dtype=torch.int32, device="cuda")
    small = ctx.load_db(rg.pir_params(), synth.db_bytes(8, 8, 8, rg.N), 8, 8)
    out2 = torch.zeros((1, 8, 2, 2, rg.N), dtype=torch.int32, device="cuda")
    with pytest.raises(pir.PirError) as ei:
        ctx.answer_batch_static([(db, 1, q, out), (small, 1, q2, out2)])
    assert ei.value.status == 4                                      # PIR_ERR_BUDGET
    assert "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert int(out.abs().sum()) == 0 and int(out2.abs().sum()) == 0   # nothing ran
    db.free()
    small.free()
