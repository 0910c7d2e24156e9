"""Host-only tests of the continuous-batching schedule (no GPU).

pir_server_simulate runs the server's own scheduling code (the circular scan
of csrc/sched.h) against a stand-in executor that records, for every query,
which slots were scanned while it was active.  These tests check the
properties the server's exactness and fairness rest on:

* every finished query met every (prime, slot) pair exactly once, also when
  the slot count is not a multiple of the range count (including range
  counts above sqrt(K N));
* a query finishes exactly n_chunks steps after its admission;
* admission is first come, first served, into the lowest free column slot,
  never more than max_batch at once, and no two active queries share a slot;
* nothing starves: with arrivals that stop, every query finishes;
* the HBM-budget admission limit (pir_server_capacity) equals the state size
  the header documents, recomputed here from the layout, and grows with the
  budget.
"""

import numpy as np
import pytest

from oracle import params as op
from paper_2606_11536_amd import pir

NONE = np.iinfo(np.uint32).max


def _check_schedule(max_batch, n_slots, n_chunks, submits):
    a_step, a_slot, f_step, cov = pir.server_simulate(max_batch, n_slots, n_chunks, submits)
    nq = len(a_step)
    submit_step = np.repeat(np.arange(len(submits)), submits)
    done = f_step != NONE
    # exactly one lap: every slot once, finishing n_chunks - 1 steps after admission
    assert (cov[done] == 1).all()
    assert (f_step[done] - a_step[done] == n_chunks - 1).all()
    # a query still running has met each slot at most once
    assert (cov[~done] <= 1).all()
    # first come, first served: admitted no earlier than submitted, in order
    adm = a_step != NONE
    assert (a_step[adm] >= submit_step[adm]).all()
    assert (np.diff(a_step[adm].astype(np.int64)) >= 0).all()
    assert adm[: adm.sum()].all(), "a later query was admitted before an earlier one"
    # at every step: at most max_batch active, each in its own slot
    for s in range(len(submits)):
        act = adm & (a_step <= s) & (~done | (f_step >= s))
        assert act.sum() <= max_batch
        slots = a_slot[act]
        assert len(np.unique(slots)) == len(slots)
        assert (slots < max_batch).all()
    return a_step, a_slot, f_step, cov, nq


@pytest.mark.parametrize("n_slots,n_chunks", [(4096, 64), (4096, 1000), (4096, 4096), (100, 7),
                                              (2048, 2047), (8192, 3), (1, 1)])
def test_every_query_meets_every_slot_once(n_slots, n_chunks):
    steps = 3 * n_chunks + 5
    submits = np.zeros(steps, dtype=np.uint32)
    submits[0] = 3
    submits[min(1, steps - 1)] += 2
    submits[n_chunks // 2] += 4
    _, _, f_step, _, nq = _check_schedule(4, n_slots, n_chunks, submits)
    assert (f_step != NONE).all(), "a query did not finish"


def test_ranges_partition_the_slots_evenly():
    # the range a step scans is [n c / m, n (c+1) / m): sizes differ by at most one
    n_slots, n_chunks = 4096, 1000
    submits = np.zeros(n_chunks, dtype=np.uint32)
    submits[0] = 1
    _, _, _, cov, _ = _check_schedule(1, n_slots, n_chunks, submits)
    assert cov.sum() == n_slots


def test_fifo_lowest_slot_and_refill():
    # eight queries at once into three slots: 0,1,2 first; as slots free (all
    # at the same step) the next three take slots 0,1,2 again, in order
    n_chunks = 5
    submits = np.zeros(40, dtype=np.uint32)
    submits[0] = 8
    a_step, a_slot, f_step, _, _ = _check_schedule(3, 50, n_chunks, submits)
    assert list(a_slot) == [0, 1, 2, 0, 1, 2, 0, 1]
    assert list(a_step) == [0, 0, 0, 5, 5, 5, 10, 10]
    assert list(f_step) == [4, 4, 4, 9, 9, 9, 14, 14]


def test_no_starvation_under_random_arrivals():
    rng = np.random.default_rng(5)
    n_chunks, max_batch = 16, 6
    submits = rng.poisson(0.35, size=600).astype(np.uint32)
    submits[-(4 * n_chunks + 200):] = 0           # arrivals stop: the queue must drain
    a_step, a_slot, f_step, _, nq = _check_schedule(max_batch, 512, n_chunks, submits)
    assert (f_step != NONE).all()
    # under load every free slot is refilled at once: a query waits only while
    # all max_batch slots are busy
    submit_step = np.repeat(np.arange(len(submits)), submits)
    for q in range(nq):
        if a_step[q] > submit_step[q]:
            s = a_step[q] - 1
            busy = ((a_step <= s) & (f_step >= s)).sum()
            assert busy == max_batch


def test_late_joiner_mid_lap():
    # a query admitted while another is half way through its lap still covers
    # every slot once, starting from the range the scan is on
    submits = np.zeros(30, dtype=np.uint32)
    submits[0] = 1
    submits[3] = 1
    a_step, a_slot, f_step, cov, _ = _check_schedule(2, 80, 8, submits)
    assert list(a_step) == [0, 3] and list(a_slot) == [0, 1]
    assert list(f_step) == [7, 10]


def test_simulate_rejects_bad_arguments():
    with pytest.raises(pir.PirError):
        pir.server_simulate(4, 10, 11, [1])            # more ranges than slots
    with pytest.raises(pir.PirError):
        pir.server_simulate(0, 10, 2, [1])
    with pytest.raises(pir.PirError):
        pir.server_simulate(4, 10, 0, [1])


def _state_bytes(K, N, R, C, mb):
    """The server's device state for max_batch mb, from the layout the header
    documents: query limbs (R_pad x 2 mb columns, 1 byte per limb, four
    limbs, 8 columns per atom), mb answers of C x 2 x K x N words, and one
    admission's NTT-form query (R x 2 x K x N words)."""
    r_pad = (R + 63) // 64 * 64
    n_cb = (2 * mb + 7) // 8
    return K * N * r_pad * n_cb * 8 * 4 + mb * C * 2 * K * N * 4 + R * 2 * K * N * 4


@pytest.mark.parametrize("log2n,K,R,C", [(11, 2, 4096, 2048), (10, 2, 100, 30), (12, 1, 3000, 7)])
def test_capacity_matches_layout(log2n, K, R, C):
    N = 1 << log2n
    params = pir.Params(log2n, op.ntt_primes(N, K))
    held = 137 << 30
    for mb in (1, 2, 5, 64, 128):
        need = _state_bytes(K, N, R, C, mb)
        got, nbytes = pir.server_capacity(params, R, C, held, held + need, 256)
        assert nbytes == _state_bytes(K, N, R, C, got)
        assert got >= mb, "a budget that fits mb slots must admit at least mb"
        assert held + _state_bytes(K, N, R, C, got) <= held + need
        if got < 256:
            assert _state_bytes(K, N, R, C, got + 1) > need
    assert pir.server_capacity(params, R, C, held, 0, 77)[0] == 77       # no cap
    assert pir.server_capacity(params, R, C, held, held + 1, 77)[0] == 0  # not even one
