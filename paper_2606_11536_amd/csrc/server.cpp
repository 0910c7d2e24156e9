// Continuous-batching server for the scan (the request loop around the
// paper's multi-client batching, Sec. 2.5, and stream-wise buffering, Sec. 4.4).
//
// The flat slot index k*N + t of the database is cut into n_chunks ranges and
// scanned round-robin, one range per step ("circular scan").  A query is
// admitted at a step boundary into a free column slot: its forward NTT runs,
// its limbs are packed into its own two columns of the shared query atoms,
// and from then on every step's scan launch covers it together with all
// other active queries.  After n_chunks steps it has met every slot exactly
// once; its answer (NTT form, held in its slot of the answer state) is then
// inverse-transformed and copied to the caller's buffer, and the slot frees.
//
// Exactness does not depend on the mix: the result for slot (k, t) of a query
// is sum_i D[i][j] * Q[i] over that query's own columns only, computed in one
// scan launch, so a query's answer is the same bytes alone or with others.
#include <map>
#include <set>

#include "ctx.h"
#include "sched.h"

using namespace pir;

struct pir_server {
  pir_ctx *ctx = nullptr;
  const pir_db *db = nullptr;
  DbDesc d{};
  uint32_t max_batch = 0, n_cb = 0;
  CircularScan sched{1, 1, 1};
  uint8_t *qatoms = nullptr;    // query atoms [K][N][n_cb][n_ib] (column block major)
  uint32_t *ans = nullptr;      // answer state, slot-major: [K N][2 max_batch C]
  uint32_t *scratch = nullptr;  // NTT-form query of an admission
  size_t qatoms_bytes = 0, ans_bytes = 0, scratch_bytes = 0;
  struct Buffers {
    const uint32_t *q;
    uint32_t *out;
  };
  std::map<uint64_t, Buffers> buffers;          // queued or active tickets
  uint64_t next_ticket = 1;
  std::map<uint64_t, hipEvent_t> done_events;   // finished, not yet reported
  std::set<uint64_t> failed;                    // drain could not be launched
};

namespace {

// Device bytes of a server's state for max_batch mb (query atoms of every
// column slot, answer state of every slot, the NTT scratch of one admission).
size_t server_bytes(uint32_t K, uint32_t N, uint32_t R, uint32_t C, uint32_t mb) {
  const size_t n_cb = (2 * (size_t)mb + kCB - 1) / kCB, n_ib = r_pad(R) / kIB;
  return (size_t)K * N * n_ib * n_cb * kAtomBytes + (size_t)mb * C * 2 * K * N * 4 +
         (size_t)R * 2 * K * N * 4;
}

// Largest batch <= max_batch whose state fits in budget - held (0 = none;
// budget 0 = no cap).
uint32_t budget_batch(size_t held, size_t budget, uint32_t K, uint32_t N, uint32_t R, uint32_t C,
                      uint32_t max_batch) {
  if (!budget) return max_batch;
  uint32_t mb = max_batch;
  while (mb >= 1 && held + server_bytes(K, N, R, C, mb) > budget) --mb;
  return mb;
}

void server_free(pir_server *s) {
  if (!s) return;
  dev_free(s->ctx, s->qatoms, s->qatoms_bytes);
  dev_free(s->ctx, s->ans, s->ans_bytes);
  dev_free(s->ctx, s->scratch, s->scratch_bytes);
  for (auto &kv : s->done_events) (void)hipEventDestroy(kv.second);
  delete s;
}

// Launch the drain of a query that met every range: its polynomials out of
// the slot-major state, the INTT in place, and a completion event.
hipError_t drain_slot(pir_server *s, uint32_t k, uint32_t *out, hipStream_t st, hipEvent_t *ev) {
  const DbDesc &d = s->d;
  hipError_t e = launch_unpack_answers(s->ans, 2 * s->max_batch * d.C, 2 * k * d.C, 2 * d.C,
                                       d.K * d.N, out, st);
  if (e == hipSuccess) e = launch_ntt(out, (size_t)d.C * 2 * d.K, d.K, d.log2n, d.primes, true, st);
  if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  if (e == hipSuccess) {
    e = hipEventRecord(*ev, st);
    if (e != hipSuccess) (void)hipEventDestroy(*ev);
  }
  return e;
}

}  // namespace

extern "C" {

pir_status pir_server_capacity(const pir_params *params, uint32_t R, uint32_t C, size_t held_bytes,
                               size_t budget_bytes, uint32_t max_batch, uint32_t *admitted,
                               size_t *state_bytes) {
  if (!params || !admitted) return fail(nullptr, PIR_ERR_INVALID_ARG, "null argument");
  pir_status st = pir_params_check(params, nullptr);
  if (st != PIR_OK) return st;
  if (R < 1 || R > PIR_MAX_R || C < 1 || C > PIR_MAX_C || max_batch < 1 ||
      max_batch > PIR_MAX_BATCH)
    return fail(nullptr, PIR_ERR_INVALID_ARG, "R, C or max_batch out of range");
  const uint32_t N = 1u << params->log2_n, K = params->n_primes;
  *admitted = budget_batch(held_bytes, budget_bytes, K, N, R, C, max_batch);
  if (state_bytes) *state_bytes = *admitted ? server_bytes(K, N, R, C, *admitted) : 0;
  return PIR_OK;
}

pir_status pir_server_simulate(uint32_t max_batch, uint32_t n_slots, uint32_t n_chunks,
                               const uint32_t *submits, uint32_t n_steps, uint32_t n_queries,
                               uint32_t *admit_step, uint32_t *admit_slot, uint32_t *finish_step,
                               uint32_t *cover) {
  if (max_batch < 1 || max_batch > PIR_MAX_BATCH || n_slots < 1 || n_chunks < 1 ||
      n_chunks > n_slots || (!submits && n_steps) || !admit_step || !admit_slot || !finish_step)
    return fail(nullptr, PIR_ERR_INVALID_ARG, "bad simulation arguments");
  uint64_t total = 0;
  for (uint32_t s = 0; s < n_steps; ++s) total += submits[s];
  if (total != n_queries) return fail(nullptr, PIR_ERR_INVALID_ARG, "submits do not sum to n_queries");
  for (uint32_t q = 0; q < n_queries; ++q) admit_step[q] = admit_slot[q] = finish_step[q] = UINT32_MAX;
  if (cover)
    for (size_t i = 0; i < (size_t)n_queries * n_slots; ++i) cover[i] = 0;
  CircularScan sc(max_batch, n_slots, n_chunks);
  uint64_t next = 0;
  for (uint32_t step = 0; step < n_steps; ++step) {
    for (uint32_t i = 0; i < submits[step]; ++i) sc.submit(next++);
    uint32_t k;
    uint64_t t;
    while (sc.next_admission(&k, &t)) {
      sc.admit(k);
      admit_step[t] = step;
      admit_slot[t] = k;
    }
    // the stand-in executor: the scan of this step's range for every active query
    if (cover && sc.b_eff()) {
      const uint32_t c = sc.chunk();
      for (uint32_t j = 0; j < sc.max_batch(); ++j)
        if (sc.slot(j).active)
          for (uint32_t x = sc.range_begin(c); x < sc.range_end(c); ++x)
            ++cover[(size_t)sc.slot(j).ticket * n_slots + x];
    }
    for (uint32_t j : sc.advance()) {
      finish_step[sc.slot(j).ticket] = step;
      sc.release(j);
    }
  }
  return PIR_OK;
}

pir_status pir_server_create(pir_ctx *ctx, const pir_db *db, uint32_t max_batch, uint32_t n_chunks,
                             pir_server **out) {
  if (!ctx || !out) return PIR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!db || db->ctx != ctx) return fail(ctx, PIR_ERR_INVALID_ARG, "bad database");
  const DbDesc &d = db->desc;
  if (max_batch < 1 || max_batch > PIR_MAX_BATCH)
    return fail(ctx, PIR_ERR_INVALID_ARG, "max_batch=%u out of range", max_batch);
  if (n_chunks < 1 || n_chunks > d.K * d.N)
    return fail(ctx, PIR_ERR_INVALID_ARG, "n_chunks=%u out of range [1, %u]", n_chunks, d.K * d.N);
  DeviceGuard g(ctx->device);
  // Admission is bounded by the HBM budget: keep the largest batch whose
  // query and answer state fit next to what the context already holds.
  const uint32_t mb = budget_batch(ctx->held, ctx->budget, d.K, d.N, d.R, d.C, max_batch);
  if (mb == 0) return fail(ctx, PIR_ERR_BUDGET, "no room for one query's state under the HBM budget");
  pir_server *s = new (std::nothrow) pir_server;
  if (!s) return fail(ctx, PIR_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->ctx = ctx;
  s->db = db;
  s->d = d;
  s->max_batch = mb;
  s->n_cb = (2 * mb + kCB - 1) / kCB;
  s->sched = CircularScan(mb, d.K * d.N, n_chunks);
  s->qatoms_bytes = (size_t)d.K * d.N * d.n_ib * s->n_cb * kAtomBytes;
  s->ans_bytes = (size_t)mb * d.C * 2 * d.K * d.N * 4;
  s->scratch_bytes = (size_t)d.R * 2 * d.K * d.N * 4;
  pir_status st;
  if ((st = dev_alloc(ctx, (void **)&s->qatoms, s->qatoms_bytes, "server query state")) != PIR_OK ||
      (st = dev_alloc(ctx, (void **)&s->ans, s->ans_bytes, "server answer state")) != PIR_OK ||
      (st = dev_alloc(ctx, (void **)&s->scratch, s->scratch_bytes, "server scratch")) != PIR_OK) {
    server_free(s);
    return st;
  }
  // columns of free slots hold zeros until a query is packed into them
  if (hipMemset(s->qatoms, 0, s->qatoms_bytes) != hipSuccess) {
    server_free(s);
    return fail(ctx, PIR_ERR_DEVICE, "hipMemset of the server query state failed");
  }
  *out = s;
  return PIR_OK;
}

void pir_server_destroy(pir_server *s) {
  if (!s) return;
  DeviceGuard g(s->ctx->device);
  (void)hipDeviceSynchronize();
  server_free(s);
}

pir_status pir_server_submit(pir_server *s, const uint32_t *query_coeff, uint32_t *answer_coeff,
                             uint64_t *ticket) {
  if (!s) return PIR_ERR_INVALID_ARG;
  if (!query_coeff || !answer_coeff || !ticket)
    return fail(s->ctx, PIR_ERR_INVALID_ARG, "null argument");
  const uint64_t t = s->next_ticket++;
  s->buffers[t] = {query_coeff, answer_coeff};
  s->sched.submit(t);
  *ticket = t;
  return PIR_OK;
}

pir_status pir_server_step(pir_server *s, pir_stream stream, uint32_t *admitted,
                           uint32_t *finished) {
  if (!s) return PIR_ERR_INVALID_ARG;
  pir_ctx *ctx = s->ctx;
  DeviceGuard g(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  const DbDesc &d = s->d;
  CircularScan &sc = s->sched;
  uint32_t n_adm = 0, n_fin = 0;
  if (admitted) *admitted = 0;
  if (finished) *finished = 0;
  // 1. admit queued queries into free column slots (oldest first, lowest slot
  // first).  A query whose launches fail stays queued, so a later step (or
  // the caller, after the error) finds the server consistent.
  uint32_t k;
  uint64_t t;
  while (sc.next_admission(&k, &t)) {
    const pir_server::Buffers &b = s->buffers.at(t);
    HIP_OR_FAIL(ctx, launch_ntt_copy(b.q, s->scratch, (size_t)d.R * 2 * d.K, d.K, d.log2n,
                                     d.primes, st));
    HIP_OR_FAIL(ctx, launch_pack_query_slot(s->scratch, s->qatoms, k, s->n_cb, d.R, d.N, d.K, st));
    sc.admit(k);
    ++n_adm;
  }
  // 2. scan this step's range for every active query; on failure the step
  // has changed nothing but admissions and may be repeated
  const uint32_t b_eff = sc.b_eff();
  if (b_eff) {
    const uint32_t slot0 = sc.range_begin(sc.chunk()), n = sc.range_end(sc.chunk()) - slot0;
    ScanJob job{d, s->qatoms, nullptr, s->ans, b_eff, slot0, n, s->n_cb, 2 * s->max_batch * d.C, 1};
    HIP_OR_FAIL(ctx, launch_scan(&job, 1, server_scan_cfg(ctx, d, b_eff), st));
  }
  // 3. queries that have now met every range finish; a drain that cannot be
  // launched marks its ticket failed (poll then reports PIR_ERR_DEVICE)
  bool drain_failed = false;
  for (uint32_t j : sc.advance()) {
    const uint64_t tk = sc.slot(j).ticket;
    hipEvent_t ev = nullptr;
    if (drain_slot(s, j, s->buffers.at(tk).out, st, &ev) == hipSuccess) {
      s->done_events[tk] = ev;
      ++n_fin;
    } else {
      s->failed.insert(tk);
      drain_failed = true;
    }
    s->buffers.erase(tk);
    sc.release(j);
  }
  if (admitted) *admitted = n_adm;
  if (finished) *finished = n_fin;
  if (drain_failed) return fail(ctx, PIR_ERR_DEVICE, "answer drain launch failed");
  return PIR_OK;
}

pir_status pir_server_poll(pir_server *s, uint64_t ticket, int *done) {
  if (!s || !done) return PIR_ERR_INVALID_ARG;
  if (s->buffers.count(ticket)) {
    *done = 0;
    return PIR_OK;
  }
  if (s->failed.erase(ticket)) {
    *done = 0;
    return fail(s->ctx, PIR_ERR_DEVICE, "ticket %llu failed: its answer drain was not launched",
                (unsigned long long)ticket);
  }
  auto it = s->done_events.find(ticket);
  if (it == s->done_events.end())
    return fail(s->ctx, PIR_ERR_INVALID_ARG, "unknown or already reported ticket %llu",
                (unsigned long long)ticket);
  DeviceGuard g(s->ctx->device);
  const hipError_t e = hipEventQuery(it->second);
  if (e == hipErrorNotReady) {
    *done = 0;
    return PIR_OK;
  }
  if (e != hipSuccess) return fail(s->ctx, PIR_ERR_DEVICE, "hipEventQuery: %s", hipGetErrorString(e));
  (void)hipEventDestroy(it->second);
  s->done_events.erase(it);
  *done = 1;
  return PIR_OK;
}

pir_status pir_server_info(const pir_server *s, uint32_t *max_batch, uint32_t *active,
                           uint32_t *queued, uint32_t *next_chunk) {
  if (!s) return PIR_ERR_INVALID_ARG;
  if (max_batch) *max_batch = s->max_batch;
  if (active) *active = s->sched.active();
  if (queued) *queued = s->sched.queued();
  if (next_chunk) *next_chunk = s->sched.chunk();
  return PIR_OK;
}

}  // extern "C"
