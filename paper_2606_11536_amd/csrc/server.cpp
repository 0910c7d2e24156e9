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
#include <deque>
#include <set>

#include "ctx.h"

using namespace pir;

struct pir_server {
  pir_ctx *ctx = nullptr;
  const pir_db *db = nullptr;
  DbDesc d{};
  uint32_t max_batch = 0, n_cb = 0, n_chunks = 0, n_slots = 0, chunk_len = 0;
  uint32_t chunk = 0;
  uint8_t *qatoms = nullptr;
  uint32_t *ans = nullptr;      // answer state, slot-major: [K N][2 max_batch C]
  uint32_t *scratch = nullptr;  // NTT-form query of an admission
  size_t qatoms_bytes = 0, ans_bytes = 0, scratch_bytes = 0;
  struct Slot {
    bool active = false;
    uint64_t ticket = 0;
    uint32_t done = 0;
    uint32_t *out = nullptr;
  };
  std::vector<Slot> slots;
  struct Pending {
    uint64_t ticket;
    const uint32_t *q;
    uint32_t *out;
  };
  std::deque<Pending> pending;
  uint64_t next_ticket = 1;
  std::set<uint64_t> in_flight;                 // queued or active
  std::map<uint64_t, hipEvent_t> done_events;   // finished, not yet reported
};

namespace {

size_t answer_bytes(const DbDesc &d) { return (size_t)d.C * 2 * d.K * d.N * 4; }

size_t server_bytes(const DbDesc &d, uint32_t mb) {
  const size_t n_cb = (2 * (size_t)mb + kCB - 1) / kCB;
  return (size_t)d.K * d.N * d.n_ib * n_cb * kAtomBytes + mb * answer_bytes(d) +
         (size_t)d.R * 2 * d.K * d.N * 4;
}

void server_free(pir_server *s) {
  if (!s) return;
  dev_free(s->ctx, s->qatoms, s->qatoms_bytes);
  dev_free(s->ctx, s->ans, s->ans_bytes);
  dev_free(s->ctx, s->scratch, s->scratch_bytes);
  for (auto &kv : s->done_events) (void)hipEventDestroy(kv.second);
  delete s;
}

}  // namespace

extern "C" {

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
  uint32_t mb = max_batch;
  if (ctx->budget) {
    while (mb >= 1 && ctx->held + server_bytes(d, mb) > ctx->budget) --mb;
    if (mb == 0)
      return fail(ctx, PIR_ERR_BUDGET, "no room for one query's state under the HBM budget");
  }
  pir_server *s = new (std::nothrow) pir_server;
  if (!s) return fail(ctx, PIR_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->ctx = ctx;
  s->db = db;
  s->d = d;
  s->max_batch = mb;
  s->n_cb = (2 * mb + kCB - 1) / kCB;
  s->n_chunks = n_chunks;
  s->n_slots = d.K * d.N;
  s->chunk_len = (s->n_slots + n_chunks - 1) / n_chunks;
  s->slots.resize(mb);
  s->qatoms_bytes = (size_t)d.K * d.N * d.n_ib * s->n_cb * kAtomBytes;
  s->ans_bytes = mb * answer_bytes(d);
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
  s->pending.push_back({t, query_coeff, answer_coeff});
  s->in_flight.insert(t);
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
  uint32_t n_adm = 0, n_fin = 0;
  // 1. admit queued queries into free column slots (lowest slot first)
  for (uint32_t k = 0; k < s->max_batch && !s->pending.empty(); ++k) {
    pir_server::Slot &sl = s->slots[k];
    if (sl.active) continue;
    const pir_server::Pending p = s->pending.front();
    s->pending.pop_front();
    HIP_OR_FAIL(ctx, launch_ntt_copy(p.q, s->scratch, (size_t)d.R * 2 * d.K, d.K, d.log2n,
                                     d.primes, st));
    HIP_OR_FAIL(ctx, launch_pack_query_slot(s->scratch, s->qatoms, k, s->n_cb, d.R, d.N, d.K, st));
    sl.active = true;
    sl.ticket = p.ticket;
    sl.done = 0;
    sl.out = p.out;
    ++n_adm;
  }
  // 2. scan this step's range of slots for every active query
  uint32_t b_eff = 0;
  for (uint32_t k = 0; k < s->max_batch; ++k)
    if (s->slots[k].active) b_eff = k + 1;
  if (b_eff) {
    const uint32_t slot0 = s->chunk * s->chunk_len;
    const uint32_t n = std::min(s->chunk_len, s->n_slots - slot0);
    ScanJob job{d, s->qatoms, nullptr, s->ans, b_eff, slot0, n, s->n_cb, 2 * s->max_batch * d.C};
    HIP_OR_FAIL(ctx, launch_scan(&job, 1, server_scan_cfg(ctx, d, b_eff), st));
    // 3. queries that have now met every range finish
    for (uint32_t k = 0; k < s->max_batch; ++k) {
      pir_server::Slot &sl = s->slots[k];
      if (!sl.active || ++sl.done < s->n_chunks) continue;
      // the slot's polynomials out of the slot-major state, then the INTT in place
      HIP_OR_FAIL(ctx, launch_unpack_answers(s->ans, 2 * s->max_batch * d.C, 2 * k * d.C, 2 * d.C,
                                             d.K * d.N, sl.out, st));
      HIP_OR_FAIL(ctx, launch_ntt(sl.out, (size_t)d.C * 2 * d.K, d.K, d.log2n, d.primes, true, st));
      hipEvent_t ev;
      HIP_OR_FAIL(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      HIP_OR_FAIL(ctx, hipEventRecord(ev, st));
      s->done_events[sl.ticket] = ev;
      s->in_flight.erase(sl.ticket);
      sl.active = false;
      ++n_fin;
    }
  }
  s->chunk = (s->chunk + 1) % s->n_chunks;
  if (admitted) *admitted = n_adm;
  if (finished) *finished = n_fin;
  return PIR_OK;
}

pir_status pir_server_poll(pir_server *s, uint64_t ticket, int *done) {
  if (!s || !done) return PIR_ERR_INVALID_ARG;
  if (s->in_flight.count(ticket)) {
    *done = 0;
    return PIR_OK;
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
  uint32_t a = 0;
  for (const auto &sl : s->slots) a += sl.active;
  if (max_batch) *max_batch = s->max_batch;
  if (active) *active = a;
  if (queued) *queued = (uint32_t)s->pending.size();
  if (next_chunk) *next_chunk = s->chunk;
  return PIR_OK;
}

}  // extern "C"
