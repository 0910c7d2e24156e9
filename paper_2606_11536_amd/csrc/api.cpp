// Host side of libpir: the C ABI declared in include/pir.h.
//
// Parameter arithmetic (prime search, roots of unity, twiddle and limb-weight
// tables) is done here on the host in exact 64-bit integer arithmetic; all
// per-element work runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"
#include "pir_internal.h"

using namespace pir;

namespace pir {

// Message of the last failure that had no context to hold it (per thread).
thread_local std::string g_noctx_err;

pir_status fail(pir_ctx *ctx, pir_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  (ctx ? ctx->err : g_noctx_err) = buf;
  return s;
}

}  // namespace pir

namespace {

// ------------------------------------------------------- number theory ----
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)((unsigned __int128)a * b % m);
}
uint64_t powmod(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = mulmod(r, b, m);
    b = mulmod(b, b, m);
    e >>= 1;
  }
  return r;
}
// Deterministic Miller-Rabin for n < 2^32 (bases 2, 3, 5, 7 suffice below 3.2e9;
// 11 and 13 added for margin).
bool is_prime_u32(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13};
  for (uint64_t p : bases)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int r = 0;
  while ((d & 1) == 0) d >>= 1, ++r;
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r; ++i) {
      x = mulmod(x, x, n);
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}
uint32_t bitrev(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; ++i) r = (r << 1) | ((x >> i) & 1);
  return r;
}
// The smallest primitive 2N-th root of unity mod q: find one root r as
// c^((q-1)/2N) for the first c that gives order 2N, then take the minimum over
// its odd powers (exactly the set of primitive 2N-th roots).
uint32_t psi_of(uint32_t N, uint32_t q) {
  uint64_t r = 0;
  for (uint64_t c = 2; c < q; ++c) {
    const uint64_t x = powmod(c, (q - 1) / (2ull * N), q);
    if (powmod(x, N, q) == q - 1) {
      r = x;
      break;
    }
  }
  const uint64_t r2 = mulmod(r, r, q);
  uint64_t best = q, x = r;
  for (uint32_t i = 0; i < N; ++i) {
    best = std::min(best, x);
    x = mulmod(x, r2, q);
  }
  return (uint32_t)best;
}
uint32_t shoup(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }

bool log2n_ok(uint32_t l) { return l >= PIR_MIN_LOG2_N && l <= PIR_MAX_LOG2_N; }

}  // namespace

namespace pir {

pir_status check_params(pir_ctx *ctx, const pir_params *p) {
  if (!p) return fail(ctx, PIR_ERR_INVALID_ARG, "params is NULL");
  if (!log2n_ok(p->log2_n))
    return fail(ctx, PIR_ERR_UNSUPPORTED, "log2_n=%u outside [%d, %d]", p->log2_n, PIR_MIN_LOG2_N,
                PIR_MAX_LOG2_N);
  if (p->n_primes < 1 || p->n_primes > PIR_MAX_PRIMES)
    return fail(ctx, PIR_ERR_UNSUPPORTED, "n_primes=%u outside [1, %d]", p->n_primes,
                PIR_MAX_PRIMES);
  if (p->plain_log2 < 1 || p->plain_log2 > 32)
    return fail(ctx, PIR_ERR_UNSUPPORTED, "plain_log2=%u outside [1, 32]", p->plain_log2);
  const uint64_t twoN = 2ull << p->log2_n;
  for (uint32_t k = 0; k < p->n_primes; ++k) {
    const uint32_t q = p->primes[k];
    if (q >= (1u << PIR_PRIME_BITS) || q % twoN != 1 || !is_prime_u32(q))
      return fail(ctx, PIR_ERR_UNSUPPORTED, "primes[%u]=%u is not a prime < 2^28 with q = 1 mod 2N",
                  k, q);
    for (uint32_t l = 0; l < k; ++l)
      if (p->primes[l] == q) return fail(ctx, PIR_ERR_INVALID_ARG, "primes[%u] repeated", k);
  }
  return PIR_OK;
}

// ------------------------------------------------------- device memory ----
pir_status dev_alloc(pir_ctx *ctx, void **p, size_t bytes, const char *what) {
  if (ctx->budget && ctx->held + bytes > ctx->budget)
    return fail(ctx, PIR_ERR_BUDGET, "%s: %zu bytes would exceed the HBM budget (%zu of %zu held)",
                what, bytes, ctx->held, ctx->budget);
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(ctx, PIR_ERR_OUT_OF_MEMORY, "%s: hipMalloc(%zu) failed", what, bytes);
  }
  ctx->held += bytes;
  return PIR_OK;
}
void dev_free(pir_ctx *ctx, void *p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  ctx->held -= bytes;
}

pir_status ensure_ws(pir_ctx *ctx, size_t bytes) {
  if (ctx->ws_bytes >= bytes) return PIR_OK;
  HIP_OR_FAIL(ctx, hipDeviceSynchronize());
  dev_free(ctx, ctx->ws, ctx->ws_bytes);
  ctx->ws = nullptr;
  ctx->ws_bytes = 0;
  const size_t want = (bytes + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1);
  pir_status st = dev_alloc(ctx, &ctx->ws, want, "workspace");
  if (st != PIR_OK) return st;
  ctx->ws_bytes = want;
  return PIR_OK;
}

}  // namespace pir

namespace pir {
// Device table of per-prime constants for (log2n, primes).
pir_status prime_set(pir_ctx *ctx, const pir_params *p, const DevPrime **out) {
  std::vector<uint32_t> key{p->log2_n};
  for (uint32_t k = 0; k < p->n_primes; ++k) key.push_back(p->primes[k]);
  auto it = ctx->prime_sets.find(key);
  if (it != ctx->prime_sets.end()) {
    *out = it->second;
    return PIR_OK;
  }
  const uint32_t N = 1u << p->log2_n;
  std::vector<DevPrime> host(p->n_primes);
  for (uint32_t k = 0; k < p->n_primes; ++k) {
    const uint32_t q = p->primes[k];
    auto tk = std::make_pair(p->log2_n, q);
    uint32_t *tw = nullptr;
    auto ti = ctx->tw_tables.find(tk);
    if (ti != ctx->tw_tables.end()) {
      tw = ti->second;
    } else {
      const uint32_t psi = psi_of(N, q);
      const uint32_t psi_inv = (uint32_t)powmod(psi, 2ull * N - 1, q);
      std::vector<uint32_t> h(4 * (size_t)N);
      for (uint32_t i = 0; i < N; ++i) {
        const uint32_t br = bitrev(i, p->log2_n);
        const uint32_t f = (uint32_t)powmod(psi, br, q), v = (uint32_t)powmod(psi_inv, br, q);
        h[i] = f;
        h[N + i] = shoup(f, q);
        h[2 * N + i] = v;
        h[3 * N + i] = shoup(v, q);
      }
      pir_status st = dev_alloc(ctx, (void **)&tw, h.size() * 4, "twiddle table");
      if (st != PIR_OK) return st;
      HIP_OR_FAIL(ctx, hipMemcpy(tw, h.data(), h.size() * 4, hipMemcpyHostToDevice));
      ctx->tw_tables[tk] = tw;
    }
    DevPrime &d = host[k];
    std::memset(&d, 0, sizeof d);
    d.q = q;
    d.log2n = p->log2_n;
    d.ninv = (uint32_t)powmod(N, q - 2, q);
    d.ninv_sh = shoup(d.ninv, q);
    for (int s = 0; s < 7; ++s) {
      d.w[s] = (uint32_t)powmod(2, 7ull * s, q);
      d.w_sh[s] = shoup(d.w[s], q);
    }
    d.tw = tw;
  }
  DevPrime *dev = nullptr;
  pir_status st = dev_alloc(ctx, (void **)&dev, sizeof(DevPrime) * host.size(), "prime table");
  if (st != PIR_OK) return st;
  HIP_OR_FAIL(ctx, hipMemcpy(dev, host.data(), sizeof(DevPrime) * host.size(), hipMemcpyHostToDevice));
  ctx->prime_sets[key] = dev;
  *out = dev;
  return PIR_OK;
}

}  // namespace pir

namespace {

// Brackets one stage launch with HIP events when profiling is on.
// Times one stage with a pair of HIP events, if that stage is being profiled:
// recorded on the stream around the stage's launches, or (attached) handed to
// a launcher through start() / stop() so that the kernel launch itself records
// them, which puts no marker commands between the kernels.
struct StageTimer {
  pir_ctx *ctx;
  hipStream_t s;
  pir_ctx::Rec rec{};
  bool on = false, attached = false;
  StageTimer(pir_ctx *c, hipStream_t st, uint32_t stage, bool attach = false, bool enabled = true)
      : ctx(c), s(st), attached(attach) {
    if (!enabled || !(ctx->prof >> stage & 1u)) return;
    rec.stage = stage;
    if (hipEventCreate(&rec.a) != hipSuccess) return;
    if (hipEventCreate(&rec.b) != hipSuccess) {
      (void)hipEventDestroy(rec.a);
      return;
    }
    on = attached || hipEventRecord(rec.a, s) == hipSuccess;
    if (!on) (void)hipEventDestroy(rec.a), (void)hipEventDestroy(rec.b);
  }
  hipEvent_t start() const { return on ? rec.a : nullptr; }
  hipEvent_t stop() const { return on ? rec.b : nullptr; }
  ~StageTimer() {
    if (!on) return;
    if (attached || hipEventRecord(rec.b, s) == hipSuccess) {
      ctx->pending.push_back(rec);
    } else {
      (void)hipEventDestroy(rec.a);
      (void)hipEventDestroy(rec.b);
    }
  }
};

void profile_drain(pir_ctx *ctx) {
  for (auto &r : ctx->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      ctx->stage_ms[r.stage] += ms;
      ctx->stage_n[r.stage] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  ctx->pending.clear();
}

// Answers of B queries: [B][C][2][K][N] words (also the slot-major size).
size_t answer_bytes(const DbDesc &d, uint32_t B) { return (size_t)B * d.C * 2 * d.K * d.N * 4; }

size_t query_atom_bytes(const DbDesc &d, uint32_t B) {
  if (B == 1) return 0;  // the batch-1 kernel reads the NTT-form query directly
  const uint32_t n_cb = (2 * B + kCB - 1) / kCB;
  return (size_t)d.K * d.N * d.n_ib * n_cb * kAtomBytes;
}

std::array<uint32_t, 5> shape_key(const DbDesc &d, uint32_t B) { return {d.N, d.K, d.R, d.C, B}; }

}  // namespace

ScanCfg pir::chosen_cfg(const pir_ctx *ctx, const DbDesc &d, uint32_t B) {
  auto it = ctx->scan_cfg.find(shape_key(d, B));
  return it != ctx->scan_cfg.end() ? it->second : scan_default(B);
}

namespace {

// Average duration of `launch` on s: one timed launch (which also warms up)
// sizes the measurement to about kTuneMs of launches, at least 3 and at most
// 50, so that variants a few percent apart are told apart also for short scans.
constexpr float kTuneMs = 5.f;

template <typename F>
hipError_t time_launches(F launch, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float *avg_ms) {
  auto timed = [&](int n, float *ms) {
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < n && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    return e;
  };
  float first = 0.f;
  hipError_t e = timed(1, &first);
  if (e != hipSuccess) return e;
  const int reps = std::min(50, std::max(3, (int)(kTuneMs / std::max(first, 1e-3f)) + 1));
  float ms = 0.f;
  e = timed(reps, &ms);
  *avg_ms = ms / reps;
  return e;
}

hipError_t run_scan(pir_ctx *ctx, const ScanJob &job, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return launch_scan(&job, 1, chosen_cfg(ctx, job.db, job.B), s, e0, e1);
}

// Key of a fused group of scan jobs: the shapes of its jobs, in order.
std::vector<uint32_t> group_key(const std::vector<ScanJob> &g) {
  std::vector<uint32_t> key{(uint32_t)g.size()};
  for (const ScanJob &j : g) {
    const auto k = shape_key(j.db, j.B);
    key.insert(key.end(), k.begin(), k.end());
  }
  return key;
}

// Variant for a fused group: the batch-tuned one, else (single job) the job's
// own choice, else the default for the group's largest batch.
ScanCfg group_cfg(const pir_ctx *ctx, const std::vector<ScanJob> &g) {
  auto it = ctx->batch_cfg.find(group_key(g));
  if (it != ctx->batch_cfg.end()) return it->second;
  if (g.size() == 1) return chosen_cfg(ctx, g[0].db, g[0].B);
  uint32_t bmax = 0;
  for (const ScanJob &j : g) bmax = std::max(bmax, j.B);
  return scan_default(bmax);
}

// Workspace layout and scan jobs of a job list (see pir_answer_batch).
struct BatchPlan {
  size_t shared_q = 0, own_q = 0, atoms = 0, slot_major = 0, switched = 0;
  std::vector<ScanJob> b1, mf;      // fused groups: batch-1 kernel, batched kernel
  std::vector<uint32_t *> qntt;     // per job: where its NTT-form query goes
  std::vector<uint8_t *> qatoms;    // per job: its query atoms (batched kernel)
  std::vector<uint32_t *> sm;       // per job: its slot-major answers (batched kernel)
  std::vector<uint32_t *> ans;      // per job: NTT-form answers before a modulus switch
  size_t bytes() const { return shared_q + own_q + atoms + slot_major + switched; }
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

pir_status plan_batch(pir_ctx *ctx, const pir_job *jobs, size_t n_jobs, BatchPlan &p) {
  for (size_t n = 0; n < n_jobs; ++n) {
    const pir_job &j = jobs[n];
    if (!j.db || !j.query_coeff || !j.answer_coeff)
      return fail(ctx, PIR_ERR_INVALID_ARG, "job %zu has a null pointer", n);
    if (j.db->ctx != ctx)
      return fail(ctx, PIR_ERR_INVALID_ARG, "job %zu: database belongs to another context", n);
    if (j.B < 1 || j.B > PIR_MAX_BATCH)
      return fail(ctx, PIR_ERR_INVALID_ARG, "job %zu: B=%u out of range", n, j.B);
    const DbDesc &d = j.db->desc;
    if (j.switch_bits > 32)
      return fail(ctx, PIR_ERR_INVALID_ARG, "job %zu: switch_bits=%u > 32", n, j.switch_bits);
    if (j.switch_bits && d.K > 2)
      return fail(ctx, PIR_ERR_UNSUPPORTED, "job %zu: modulus switching takes 1 or 2 primes", n);
    if (j.switch_bits) p.switched += al256((size_t)j.B * d.C * 2 * d.K * d.N * 4);
    const size_t qb = al256((size_t)j.B * d.R * 2 * d.K * d.N * 4);
    if (j.B == 1) p.own_q += qb;
    else p.shared_q = std::max(p.shared_q, qb);
    p.atoms += al256(query_atom_bytes(d, j.B));
    if (j.B > 1) p.slot_major += al256(answer_bytes(d, j.B));
  }
  return PIR_OK;
}

// Assign workspace regions (base = workspace) and build the scan groups.
void place_batch(const pir_job *jobs, size_t n_jobs, uint8_t *base, BatchPlan &p) {
  uint8_t *own = base + p.shared_q;
  uint8_t *atoms = own + p.own_q;
  uint8_t *sm = atoms + p.atoms;
  uint8_t *sw = sm + p.slot_major;
  p.qntt.assign(n_jobs, nullptr);
  p.qatoms.assign(n_jobs, nullptr);
  p.sm.assign(n_jobs, nullptr);
  p.ans.assign(n_jobs, nullptr);
  p.b1.clear();
  p.mf.clear();
  for (size_t n = 0; n < n_jobs; ++n) {
    const pir_job &j = jobs[n];
    const DbDesc &d = j.db->desc;
    p.qntt[n] = (uint32_t *)base;
    if (j.B == 1) {
      p.qntt[n] = (uint32_t *)own;
      own += al256((size_t)d.R * 2 * d.K * d.N * 4);
    }
    p.qatoms[n] = atoms;
    atoms += al256(query_atom_bytes(d, j.B));
    if (j.B > 1) {
      p.sm[n] = (uint32_t *)sm;
      sm += al256(answer_bytes(d, j.B));
    }
    // NTT-form answers: in place in answer_coeff, or in the workspace when the
    // drain switches them into answer_coeff
    p.ans[n] = j.answer_coeff;
    if (j.switch_bits) {
      p.ans[n] = (uint32_t *)sw;
      sw += al256((size_t)j.B * d.C * 2 * d.K * d.N * 4);
    }
    const ScanJob sj{d, p.qatoms[n], p.qntt[n], j.B == 1 ? p.ans[n] : p.sm[n], j.B, 0,
                     d.K * d.N, 0, 0};
    (j.B == 1 ? p.b1 : p.mf).push_back(sj);
  }
}

}  // namespace

// ===================================================================== ABI ==
extern "C" {

const char *pir_status_string(pir_status s) {
  switch (s) {
    case PIR_OK: return "PIR_OK";
    case PIR_ERR_INVALID_ARG: return "PIR_ERR_INVALID_ARG";
    case PIR_ERR_UNSUPPORTED: return "PIR_ERR_UNSUPPORTED";
    case PIR_ERR_OUT_OF_MEMORY: return "PIR_ERR_OUT_OF_MEMORY";
    case PIR_ERR_BUDGET: return "PIR_ERR_BUDGET";
    case PIR_ERR_DEVICE: return "PIR_ERR_DEVICE";
    case PIR_ERR_NOT_READY: return "PIR_ERR_NOT_READY";
  }
  return "PIR_ERR_UNKNOWN";
}

const char *pir_version(void) { return "libpir 0.1 (gfx950)"; }

pir_status pir_find_primes(uint32_t log2_n, uint32_t count, uint32_t bound_log2, uint32_t *out) {
  if (!out || count == 0 || log2_n > 20 || bound_log2 > 31 || bound_log2 <= log2_n + 1)
    return PIR_ERR_INVALID_ARG;
  const uint64_t step = 2ull << log2_n;
  uint64_t q = ((1ull << bound_log2) - 2) / step * step + 1;
  uint32_t found = 0;
  while (found < count && q > step) {
    if (is_prime_u32(q)) out[found++] = (uint32_t)q;
    q -= step;
  }
  return found == count ? PIR_OK : PIR_ERR_INVALID_ARG;
}

pir_status pir_params_check(const pir_params *params, uint32_t *psi_out) {
  pir_status st = check_params(nullptr, params);
  if (st != PIR_OK) return st;
  if (psi_out)
    for (uint32_t k = 0; k < params->n_primes; ++k)
      psi_out[k] = psi_of(1u << params->log2_n, params->primes[k]);
  return PIR_OK;
}

pir_status pir_ctx_create(int device, size_t hbm_budget_bytes, pir_ctx **out) {
  if (!out) return fail(nullptr, PIR_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(nullptr, PIR_ERR_DEVICE, "hipGetDeviceCount failed: %s", hipGetErrorString(e));
  }
  if (device < 0 || device >= n)
    return fail(nullptr, PIR_ERR_DEVICE, "device %d not present (%d devices)", device, n);
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess)
    return fail(nullptr, PIR_ERR_DEVICE, "hipDeviceGetAttribute failed: %s", hipGetErrorString(e));
  pir_ctx *ctx = new (std::nothrow) pir_ctx;
  if (!ctx) return fail(nullptr, PIR_ERR_OUT_OF_MEMORY, "host allocation failed");
  ctx->device = device;
  ctx->budget = hbm_budget_bytes;
  ctx->num_cus = cus;
  {
    // the device address of the fixed scratch array (pir_answer_batch_static),
    // taken once per device with that device current
    DeviceGuard g(device);
    e = static_scratch_init(device, &ctx->scratch);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      ctx->scratch = nullptr;
      ctx->scratch_err = hipGetErrorString(e);
    }
  }
  *out = ctx;
  return PIR_OK;
}

void pir_ctx_destroy(pir_ctx *ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  profile_drain(ctx);
  dev_free(ctx, ctx->ws, ctx->ws_bytes);
  for (auto &kv : ctx->prime_sets) (void)hipFree(kv.second);
  for (auto &kv : ctx->tw_tables) (void)hipFree(kv.second);
  delete ctx;
}

const char *pir_last_error(const pir_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_noctx_err.c_str();
}

size_t pir_ctx_device_bytes(const pir_ctx *ctx) { return ctx ? ctx->held : 0; }

pir_status pir_ctx_reserve(pir_ctx *ctx, size_t bytes) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  DeviceGuard g(ctx->device);
  return ensure_ws(ctx, bytes);
}

}  // extern "C"

namespace {

// Lift, transform and tile R x C polynomials into a new database.
// lift(i0, valid, S, tmp) launches the lift + NTT of slab rows [i0, i0 + S)
// (rows >= i0 + valid zero) into tmp ([K][S][C][N]); after each slab the
// rows are packed into the scan atoms.
template <typename Lift>
pir_status load_rows(pir_ctx *ctx, const pir_params *params, uint32_t R, uint32_t C, hipStream_t s,
                     Lift lift, pir_db **out) {
  const DevPrime *primes = nullptr;
  pir_status st = prime_set(ctx, params, &primes);
  if (st != PIR_OK) return st;
  const uint32_t N = 1u << params->log2_n, K = params->n_primes;
  const uint32_t Rp = r_pad(R), Cp = c_pad(C);
  // + a tail: the batched kernel's padded contraction steps read past the
  // last atom of the last slot (their products meet zero query atoms)
  const size_t bytes = (size_t)K * N * Rp * Cp * 4 + kDbTailBytes;
  pir_db *db = new (std::nothrow) pir_db;
  if (!db) return fail(ctx, PIR_ERR_OUT_OF_MEMORY, "host allocation failed");
  db->ctx = ctx;
  db->params = *params;
  db->R = R;
  db->C = C;
  db->bytes = bytes;
  if ((st = dev_alloc(ctx, (void **)&db->atoms, bytes, "database")) != PIR_OK) {
    delete db;
    return st;
  }
  // Slab of S rows (multiple of 32) with a temporary NTT-form buffer of ~256 MiB.
  const size_t row_bytes = (size_t)K * C * N * 4;
  uint32_t S = (uint32_t)std::max<size_t>(32, ((256u << 20) / row_bytes) / 32 * 32);
  S = std::min(S, Rp);
  uint32_t *tmp = nullptr;
  const size_t tmp_bytes = (size_t)S * row_bytes;
  auto cleanup = [&](pir_status code) {
    (void)hipStreamSynchronize(s);
    dev_free(ctx, tmp, tmp_bytes);
    if (code != PIR_OK) {
      dev_free(ctx, db->atoms, db->bytes);
      delete db;
    }
    return code;
  };
  if ((st = dev_alloc(ctx, (void **)&tmp, tmp_bytes, "load slab")) != PIR_OK) return cleanup(st);
  for (uint32_t i0 = 0; i0 < Rp; i0 += S) {
    const uint32_t valid = i0 < R ? std::min(S, R - i0) : 0;
    if ((st = lift(i0, valid, S, tmp, primes)) != PIR_OK) return cleanup(st);
    const hipError_t e = launch_pack_db(tmp, db->atoms, i0, S, R, C, N, K, s);
    if (e != hipSuccess)
      return cleanup(fail(ctx, PIR_ERR_DEVICE, "DB transform launch failed: %s", hipGetErrorString(e)));
  }
  if (hipStreamSynchronize(s) != hipSuccess)
    return cleanup(fail(ctx, PIR_ERR_DEVICE, "DB transform failed"));
  DbDesc &d = db->desc;
  d.atoms = db->atoms;
  d.primes = primes;
  d.R = R;
  d.C = C;
  d.N = N;
  d.K = K;
  d.log2n = params->log2_n;
  d.n_jb = Cp / kJB;
  d.n_ib = Rp / kIB;
  *out = db;
  return cleanup(PIR_OK);
}

}  // namespace

extern "C" {

pir_status pir_db_load_ntt(pir_ctx *ctx, const pir_params *params, const uint8_t *raw,
                           int raw_is_device, uint32_t R, uint32_t C, pir_stream stream,
                           pir_db **out) {
  if (!ctx || !out) return PIR_ERR_INVALID_ARG;
  *out = nullptr;
  pir_status st = check_params(ctx, params);
  if (st != PIR_OK) return st;
  if (!raw) return fail(ctx, PIR_ERR_INVALID_ARG, "raw is NULL");
  if (R < 1 || R > PIR_MAX_R || C < 1 || C > PIR_MAX_C)
    return fail(ctx, PIR_ERR_INVALID_ARG, "R=%u or C=%u out of range", R, C);
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const uint32_t N = 1u << params->log2_n, K = params->n_primes;
  uint8_t *stage = nullptr;
  size_t stage_bytes = 0;
  if (!raw_is_device) {
    const size_t row_bytes = (size_t)K * C * N * 4;
    const uint32_t S = std::min((uint32_t)std::max<size_t>(32, ((256u << 20) / row_bytes) / 32 * 32),
                                r_pad(R));
    stage_bytes = (size_t)S * C * N;
    if ((st = dev_alloc(ctx, (void **)&stage, stage_bytes, "load staging")) != PIR_OK) return st;
  }
  auto lift = [&](uint32_t i0, uint32_t valid, uint32_t S, uint32_t *tmp, const DevPrime *primes) {
    const uint8_t *src = raw + (size_t)i0 * C * N;
    if (!raw_is_device && valid) {
      if (S * (size_t)C * N > stage_bytes ||
          hipMemcpyAsync(stage, src, (size_t)valid * C * N, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(ctx, PIR_ERR_DEVICE, "host-to-device copy of the raw DB failed");
      src = stage;
    }
    const hipError_t e = launch_lift_ntt(valid ? src : nullptr, tmp, S, valid, C, K,
                                         params->log2_n, primes, s);
    return e == hipSuccess ? PIR_OK
                           : fail(ctx, PIR_ERR_DEVICE, "DB transform launch failed: %s",
                                  hipGetErrorString(e));
  };
  st = load_rows(ctx, params, R, C, s, lift, out);
  (void)hipStreamSynchronize(s);
  dev_free(ctx, stage, stage_bytes);
  return st;
}

pir_status pir_pack_load(pir_ctx *ctx, const pir_params *params, const uint32_t *A, int a_is_device,
                         uint32_t D1, uint32_t n, pir_stream stream, pir_db **out) {
  if (!ctx || !out) return PIR_ERR_INVALID_ARG;
  *out = nullptr;
  pir_status st = check_params(ctx, params);
  if (st != PIR_OK) return st;
  if (!A) return fail(ctx, PIR_ERR_INVALID_ARG, "A is NULL");
  const uint32_t N = 1u << params->log2_n;
  const uint32_t Cp = (uint32_t)(((uint64_t)D1 + N - 1) / N);
  if (D1 < 1 || n < 1 || n > PIR_MAX_R || Cp > PIR_MAX_C)
    return fail(ctx, PIR_ERR_INVALID_ARG, "D1=%u or n=%u out of range", D1, n);
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const size_t a_bytes = (size_t)D1 * n * 4, at_bytes = (size_t)n * Cp * N * 4;
  uint32_t *a_dev = nullptr, *at = nullptr;
  auto done = [&](pir_status code) {
    (void)hipStreamSynchronize(s);
    if (!a_is_device) dev_free(ctx, a_dev, a_bytes);
    dev_free(ctx, at, at_bytes);
    return code;
  };
  if (a_is_device) {
    a_dev = const_cast<uint32_t *>(A);
  } else {
    if ((st = dev_alloc(ctx, (void **)&a_dev, a_bytes, "LWE matrix staging")) != PIR_OK)
      return done(st);
    if (hipMemcpyAsync(a_dev, A, a_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
      return done(fail(ctx, PIR_ERR_DEVICE, "host-to-device copy of the LWE matrix failed"));
  }
  // A [D1][n] -> AT [n][Cp N]: row i of AT holds column i of A, so that
  // polynomial (i, r) (coefficient j = A[r N + j][i]) is AT[i][r N .. r N + N)
  if ((st = dev_alloc(ctx, (void **)&at, at_bytes, "LWE matrix transpose")) != PIR_OK)
    return done(st);
  if (launch_transpose32(a_dev, at, D1, n, Cp * N, s) != hipSuccess)
    return done(fail(ctx, PIR_ERR_DEVICE, "transpose launch failed"));
  auto lift = [&](uint32_t i0, uint32_t valid, uint32_t S, uint32_t *tmp, const DevPrime *primes) {
    const hipError_t e = launch_lift_ntt32(valid ? at + (size_t)i0 * Cp * N : nullptr, tmp, S, valid,
                                           Cp, params->n_primes, params->log2_n, primes, s);
    return e == hipSuccess ? PIR_OK
                           : fail(ctx, PIR_ERR_DEVICE, "hint transform launch failed: %s",
                                  hipGetErrorString(e));
  };
  st = load_rows(ctx, params, n, Cp, s, lift, out);
  if (st == PIR_OK) (*out)->pack_d1 = D1;
  return done(st);
}

pir_status pir_db_info(const pir_db *db, pir_params *params, uint32_t *R, uint32_t *C,
                       size_t *device_bytes) {
  if (!db) return PIR_ERR_INVALID_ARG;
  if (params) *params = db->params;
  if (R) *R = db->R;
  if (C) *C = db->C;
  if (device_bytes) *device_bytes = db->bytes;
  return PIR_OK;
}

pir_status pir_db_read_ntt(pir_ctx *ctx, const pir_db *db, uint32_t i0, uint32_t ni,
                           uint32_t j0, uint32_t nj, uint32_t *out, pir_stream stream) {
  if (!ctx || !db || !out) return fail(ctx, PIR_ERR_INVALID_ARG, "null argument");
  if (db->ctx != ctx) return fail(ctx, PIR_ERR_INVALID_ARG, "database belongs to another context");
  if ((uint64_t)i0 + ni > db->R || (uint64_t)j0 + nj > db->C)
    return fail(ctx, PIR_ERR_INVALID_ARG, "rows/columns out of range");
  DeviceGuard g(ctx->device);
  HIP_OR_FAIL(ctx, launch_read_db(db->desc, i0, ni, j0, nj, out, (hipStream_t)stream));
  return PIR_OK;
}

void pir_db_free(pir_db *db) {
  if (!db) return;
  DeviceGuard g(db->ctx->device);
  (void)hipDeviceSynchronize();
  dev_free(db->ctx, db->atoms, db->bytes);
  delete db;
}

static pir_status ntt_common(pir_ctx *ctx, const pir_params *params, uint32_t *polys,
                             size_t n_polys, pir_stream stream, bool inverse) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  pir_status st = check_params(ctx, params);
  if (st != PIR_OK) return st;
  if (!polys && n_polys) return fail(ctx, PIR_ERR_INVALID_ARG, "polys is NULL");
  if (n_polys > (size_t)0x7fffffff / params->n_primes)
    return fail(ctx, PIR_ERR_INVALID_ARG, "too many polynomials");
  DeviceGuard g(ctx->device);
  const DevPrime *primes = nullptr;
  if ((st = prime_set(ctx, params, &primes)) != PIR_OK) return st;
  HIP_OR_FAIL(ctx, launch_ntt(polys, n_polys * params->n_primes, params->n_primes, params->log2_n,
                              primes, inverse, (hipStream_t)stream));
  return PIR_OK;
}

pir_status pir_ntt(pir_ctx *ctx, const pir_params *params, uint32_t *polys, size_t n_polys,
                   pir_stream stream) {
  return ntt_common(ctx, params, polys, n_polys, stream, false);
}

pir_status pir_intt(pir_ctx *ctx, const pir_params *params, uint32_t *polys, size_t n_polys,
                    pir_stream stream) {
  return ntt_common(ctx, params, polys, n_polys, stream, true);
}

pir_status pir_sdb_load(pir_ctx *ctx, const int8_t *db, int db_is_device, uint32_t D1,
                        uint32_t D0, pir_stream stream, pir_sdb **out) {
  if (!ctx || !out) return PIR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!db) return fail(ctx, PIR_ERR_INVALID_ARG, "db is NULL");
  if (D1 < 1 || D1 > PIR_SDB_MAX_D1 || D0 < 1 || D0 > PIR_SDB_MAX_D0)
    return fail(ctx, PIR_ERR_INVALID_ARG, "D1=%u or D0=%u out of range", D1, D0);
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const uint32_t n_rb = (D1 + 31) / 32, n_kb = ((D0 + 31) / 32 + 7) / 8 * 8;
  if ((size_t)n_rb * n_kb > ((size_t)1 << 30))  // atom indices stay 32-bit
    return fail(ctx, PIR_ERR_INVALID_ARG, "D1=%u x D0=%u is more than 2^40 bytes of tiles", D1, D0);
  const size_t bytes = (size_t)n_rb * n_kb * kAtomBytes;
  pir_sdb *h = new (std::nothrow) pir_sdb;
  if (!h) return fail(ctx, PIR_ERR_OUT_OF_MEMORY, "host allocation failed");
  void *atoms = nullptr;
  pir_status st = dev_alloc(ctx, &atoms, bytes, "scalar database");
  if (st != PIR_OK) {
    delete h;
    return st;
  }
  const int8_t *src = db;
  void *staging = nullptr;
  const size_t raw = (size_t)D1 * D0;
  auto bail = [&](pir_status code) {
    dev_free(ctx, staging, raw);
    dev_free(ctx, atoms, bytes);
    delete h;
    return code;
  };
  if (!db_is_device) {
    if ((st = dev_alloc(ctx, &staging, raw, "scalar database staging")) != PIR_OK) return bail(st);
    if (hipMemcpyAsync(staging, db, raw, hipMemcpyHostToDevice, s) != hipSuccess)
      return bail(fail(ctx, PIR_ERR_DEVICE, "host copy failed"));
    src = (const int8_t *)staging;
  }
  if (launch_sdb_pack(src, (uint8_t *)atoms, D1, D0, n_rb, n_kb, s) != hipSuccess)
    return bail(fail(ctx, PIR_ERR_DEVICE, "database pack failed"));
  if (staging) {
    if (hipStreamSynchronize(s) != hipSuccess)
      return bail(fail(ctx, PIR_ERR_DEVICE, "stream synchronisation failed"));
    dev_free(ctx, staging, raw);
    staging = nullptr;
  }
  h->ctx = ctx;
  h->D1 = D1;
  h->D0 = D0;
  h->n_rb = n_rb;
  h->n_kb = n_kb;
  h->bytes = bytes;
  h->atoms = (uint8_t *)atoms;
  *out = h;
  return PIR_OK;
}

pir_status pir_sdb_mul(pir_ctx *ctx, const pir_sdb *db, const uint32_t *query, uint32_t B,
                       uint32_t *out, pir_stream stream) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  if (!db || !query || !out) return fail(ctx, PIR_ERR_INVALID_ARG, "null argument");
  if (db->ctx != ctx) return fail(ctx, PIR_ERR_INVALID_ARG, "database belongs to another context");
  if (B < 1 || B > PIR_MAX_BATCH) return fail(ctx, PIR_ERR_INVALID_ARG, "B=%u out of range", B);
  DeviceGuard g(ctx->device);
  const uint32_t n_cb = ((B + 7) / 8 + 3) / 4 * 4;
  pir_status st = ensure_ws(ctx, (size_t)db->n_kb * n_cb * kAtomBytes);
  if (st != PIR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  uint8_t *qa = (uint8_t *)ctx->ws;
  {
    StageTimer tm(ctx, s, PIR_STAGE_PACK);
    HIP_OR_FAIL(ctx, launch_sq_pack(query, qa, B, db->D0, db->n_kb, n_cb, s));
  }
  StageTimer tm(ctx, s, PIR_STAGE_SCAN, true);
  HIP_OR_FAIL(ctx, launch_sgemm(db->atoms, qa, out, db->D1, B, db->n_rb, db->n_kb, n_cb, s,
                                tm.start(), tm.stop()));
  return PIR_OK;
}

void pir_sdb_free(pir_sdb *db) {
  if (!db) return;
  DeviceGuard g(db->ctx->device);
  (void)hipDeviceSynchronize();
  dev_free(db->ctx, db->atoms, db->bytes);
  delete db;
}

pir_status pir_intt_modswitch(pir_ctx *ctx, const pir_params *params, const uint32_t *answer_ntt,
                              size_t n_polys, uint32_t bits, uint32_t *out, pir_stream stream) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  pir_status st = check_params(ctx, params);
  if (st != PIR_OK) return st;
  if (params->n_primes > 2)
    return fail(ctx, PIR_ERR_UNSUPPORTED, "modulus switching takes 1 or 2 primes, not %u",
                params->n_primes);
  if (bits < 1 || bits > 32) return fail(ctx, PIR_ERR_INVALID_ARG, "bits=%u not in [1, 32]", bits);
  if ((!answer_ntt || !out) && n_polys) return fail(ctx, PIR_ERR_INVALID_ARG, "null buffer");
  if (n_polys > (size_t)0x7fffffff) return fail(ctx, PIR_ERR_INVALID_ARG, "too many polynomials");
  if (n_polys == 0) return PIR_OK;
  DeviceGuard g(ctx->device);
  const DevPrime *primes = nullptr;
  if ((st = prime_set(ctx, params, &primes)) != PIR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  StageTimer tm(ctx, s, PIR_STAGE_INTT);
  HIP_OR_FAIL(ctx, launch_intt_switch(answer_ntt, out, n_polys, params->n_primes, params->primes,
                                      params->log2_n, primes, bits, s));
  return PIR_OK;
}

pir_status pir_db_mul(pir_ctx *ctx, const pir_db *db, const uint32_t *query_ntt, uint32_t B,
                      uint32_t *answer_ntt, pir_stream stream) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  if (!db || !query_ntt || !answer_ntt) return fail(ctx, PIR_ERR_INVALID_ARG, "null argument");
  if (db->ctx != ctx) return fail(ctx, PIR_ERR_INVALID_ARG, "database belongs to another context");
  if (B < 1 || B > PIR_MAX_BATCH) return fail(ctx, PIR_ERR_INVALID_ARG, "B=%u out of range", B);
  DeviceGuard g(ctx->device);
  const DbDesc &d = db->desc;
  // B > 1: query atoms, then the slot-major answers of the batched kernel
  const size_t qa = B > 1 ? al256(query_atom_bytes(d, B)) : 0;
  const size_t sm = B > 1 ? answer_bytes(d, B) : 0;
  pir_status st = ensure_ws(ctx, std::max<size_t>(qa + sm, 256));
  if (st != PIR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  uint8_t *qatoms = (uint8_t *)ctx->ws;
  uint32_t *slot_major = (uint32_t *)((uint8_t *)ctx->ws + qa);
  if (B > 1) {
    StageTimer tm(ctx, s, PIR_STAGE_PACK);
    HIP_OR_FAIL(ctx, launch_pack_query(query_ntt, qatoms, B, db->R, d.N, d.K, s));
  }
  ScanJob job{d, qatoms, query_ntt, B > 1 ? slot_major : answer_ntt, B, 0, d.K * d.N, 0, 0};
  {
    StageTimer tm(ctx, s, PIR_STAGE_SCAN, true);
    HIP_OR_FAIL(ctx, run_scan(ctx, job, s, tm.start(), tm.stop()));
  }
  if (B > 1) {
    StageTimer tm(ctx, s, PIR_STAGE_UNPACK);
    const uint32_t P = 2 * B * d.C;
    HIP_OR_FAIL(ctx, launch_unpack_answers(slot_major, P, 0, P, d.K * d.N, answer_ntt, s));
  }
  return PIR_OK;
}

}  // extern "C"

namespace {

// Enqueue the whole batch (NTT, packing, fused scans, INTT) on `s` using the
// workspace at `ws` (at least p.bytes()).
// add (may be null): per job, an addend for the component-1 answer
// polynomials ([B][C][K][N], NTT form) taken in by the drain (ring packing).
// timed = false: no stage timers (they create events), for the no-allocation entry.
pir_status enqueue_batch(pir_ctx *ctx, const pir_job *jobs, size_t n_jobs, uint8_t *ws,
                         BatchPlan &p, hipStream_t s, const uint32_t *const *add = nullptr,
                         bool timed = true) {
  place_batch(jobs, n_jobs, ws, p);
  for (size_t n = 0; n < n_jobs; ++n) {
    const pir_job &j = jobs[n];
    const DbDesc &d = j.db->desc;
    {
      StageTimer tm(ctx, s, PIR_STAGE_NTT, false, timed);
      HIP_OR_FAIL(ctx, launch_ntt_copy(j.query_coeff, p.qntt[n], (size_t)j.B * d.R * 2 * d.K, d.K,
                                       d.log2n, d.primes, s));
    }
    if (j.B > 1) {
      StageTimer tm(ctx, s, PIR_STAGE_PACK, false, timed);
      HIP_OR_FAIL(ctx, launch_pack_query(p.qntt[n], p.qatoms[n], j.B, d.R, d.N, d.K, s));
    }
  }
  // the scans of all jobs: one fused launch per kernel kind
  for (const std::vector<ScanJob> *grp : {&p.b1, &p.mf}) {
    if (grp->empty()) continue;
    StageTimer tm(ctx, s, PIR_STAGE_SCAN, true, timed);
    HIP_OR_FAIL(ctx, launch_scan(grp->data(), grp->size(), group_cfg(ctx, *grp), s, tm.start(),
                                 tm.stop()));
  }
  for (size_t n = 0; n < n_jobs; ++n) {
    const DbDesc &d = jobs[n].db->desc;
    if (p.sm[n]) {
      StageTimer tm(ctx, s, PIR_STAGE_UNPACK, false, timed);
      const uint32_t P = 2 * jobs[n].B * d.C;
      HIP_OR_FAIL(ctx, launch_unpack_answers(p.sm[n], P, 0, P, d.K * d.N, p.ans[n], s));
    }
    StageTimer tm(ctx, s, PIR_STAGE_INTT, false, timed);
    const uint32_t *a = add ? add[n] : nullptr;
    if (jobs[n].switch_bits) {
      HIP_OR_FAIL(ctx, launch_intt_switch(p.ans[n], jobs[n].answer_coeff,
                                          (size_t)jobs[n].B * d.C * 2, d.K,
                                          jobs[n].db->params.primes, d.log2n, d.primes,
                                          jobs[n].switch_bits, s, a));
    } else {
      HIP_OR_FAIL(ctx, launch_ntt(jobs[n].answer_coeff, (size_t)jobs[n].B * d.C * 2 * d.K, d.K,
                                  d.log2n, d.primes, true, s, a));
    }
  }
  return PIR_OK;
}

}  // namespace

struct pir_plan {
  pir_ctx *ctx = nullptr;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

pir_status pir_answer_batch(pir_ctx *ctx, const pir_job *jobs, size_t n_jobs, pir_stream stream) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  if (!jobs && n_jobs) return fail(ctx, PIR_ERR_INVALID_ARG, "jobs is NULL");
  // Workspace: one shared region for the NTT-form queries of batched jobs
  // (consumed by their pack before the next job's NTT), a region of its own
  // for each batch-1 job (read by its scan), and the query atoms of every job.
  BatchPlan p;
  pir_status st = plan_batch(ctx, jobs, n_jobs, p);
  if (st != PIR_OK || n_jobs == 0) return st;
  DeviceGuard g(ctx->device);
  if ((st = ensure_ws(ctx, p.bytes())) != PIR_OK) return st;
  return enqueue_batch(ctx, jobs, n_jobs, (uint8_t *)ctx->ws, p, (hipStream_t)stream);
}

pir_status pir_answer_batch_static(pir_ctx *ctx, const pir_job *jobs, size_t n_jobs,
                                   pir_stream stream) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  if (!jobs && n_jobs) return fail(ctx, PIR_ERR_INVALID_ARG, "jobs is NULL");
  // the same workspace layout as pir_answer_batch, placed in the fixed array
  BatchPlan p;
  pir_status st = plan_batch(ctx, jobs, n_jobs, p);
  if (st != PIR_OK || n_jobs == 0) return st;
  if (!ctx->scratch)
    return fail(ctx, PIR_ERR_DEVICE, "the static scratch array has no device address: %s",
                ctx->scratch_err.c_str());
  if (p.bytes() > kStaticScratchBytes)
    return fail(ctx, PIR_ERR_BUDGET,
                "the job list needs %zu bytes of workspace; the static scratch array holds %zu",
                p.bytes(), kStaticScratchBytes);
  DeviceGuard g(ctx->device);
  return enqueue_batch(ctx, jobs, n_jobs, (uint8_t *)ctx->scratch, p, (hipStream_t)stream,
                       nullptr, false);
}

pir_status pir_pack(pir_ctx *ctx, const pir_db *H, uint32_t B, const uint32_t *special_coeff,
                    const uint32_t *lwe_b, uint32_t *out, uint32_t switch_bits, pir_stream stream) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  if (!H || !special_coeff || !lwe_b || !out) return fail(ctx, PIR_ERR_INVALID_ARG, "null argument");
  if (H->ctx != ctx) return fail(ctx, PIR_ERR_INVALID_ARG, "hint belongs to another context");
  if (!H->pack_d1) return fail(ctx, PIR_ERR_INVALID_ARG, "not a ring-packing hint (pir_pack_load)");
  const pir_job job{H, B, special_coeff, out, switch_bits};
  BatchPlan p;
  pir_status st = plan_batch(ctx, &job, 1, p);   // checks B and switch_bits
  if (st != PIR_OK) return st;
  const DbDesc &d = H->desc;
  // Delta = floor(Q / p) mod q_k, Q = prod q_k < 2^112
  unsigned __int128 Q = 1;
  for (uint32_t k = 0; k < d.K; ++k) Q *= H->params.primes[k];
  const unsigned __int128 delta = Q >> H->params.plain_log2;
  uint32_t dk[PIR_MAX_PRIMES] = {};
  for (uint32_t k = 0; k < d.K; ++k) dk[k] = (uint32_t)(delta % H->params.primes[k]);
  DeviceGuard g(ctx->device);
  const size_t g_bytes = al256((size_t)B * d.C * d.K * d.N * 4);
  if ((st = ensure_ws(ctx, p.bytes() + g_bytes)) != PIR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  uint32_t *gmat = (uint32_t *)((uint8_t *)ctx->ws + p.bytes());
  {
    StageTimer tm(ctx, s, PIR_STAGE_NTT);
    HIP_OR_FAIL(ctx, launch_offset_ntt(lwe_b, gmat, B, H->pack_d1, d.C, d.K, d.log2n, d.primes, dk,
                                       s));
  }
  const uint32_t *add[1] = {gmat};
  return enqueue_batch(ctx, &job, 1, (uint8_t *)ctx->ws, p, s, add);
}

pir_status pir_plan_create(pir_ctx *ctx, const pir_job *jobs, size_t n_jobs, pir_stream stream,
                           pir_plan **out) {
  if (!ctx || !out) return PIR_ERR_INVALID_ARG;
  *out = nullptr;
  if (!jobs || n_jobs == 0) return fail(ctx, PIR_ERR_INVALID_ARG, "no jobs");
  BatchPlan p;
  pir_status st = plan_batch(ctx, jobs, n_jobs, p);
  if (st != PIR_OK) return st;
  DeviceGuard g(ctx->device);
  pir_plan *pl = new (std::nothrow) pir_plan;
  if (!pl) return fail(ctx, PIR_ERR_OUT_OF_MEMORY, "host allocation failed");
  pl->ctx = ctx;
  pl->ws_bytes = std::max<size_t>(p.bytes(), 256);
  auto bail = [&](pir_status code) {
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    dev_free(ctx, pl->ws, pl->ws_bytes);
    delete pl;
    return code;
  };
  if ((st = dev_alloc(ctx, &pl->ws, pl->ws_bytes, "plan workspace")) != PIR_OK) return bail(st);
  // Capture on a private stream (kernel launches only; no timing events).
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(ctx, PIR_ERR_DEVICE, "hipStreamCreate failed"));
  const uint32_t prof = ctx->prof;
  ctx->prof = 0;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  pir_status qst = PIR_OK;
  if (e == hipSuccess) qst = enqueue_batch(ctx, jobs, n_jobs, (uint8_t *)pl->ws, p, cs);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(cs, &graph) : e;
  ctx->prof = prof;
  (void)hipStreamDestroy(cs);
  pl->graph = graph;
  if (qst != PIR_OK) return bail(qst);
  if (e != hipSuccess || e2 != hipSuccess || !graph)
    return bail(fail(ctx, PIR_ERR_DEVICE, "graph capture failed: %s",
                     hipGetErrorString(e != hipSuccess ? e : e2)));
  if ((e = hipGraphInstantiate(&pl->exec, graph, nullptr, nullptr, 0)) != hipSuccess)
    return bail(fail(ctx, PIR_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e)));
  (void)stream;
  *out = pl;
  return PIR_OK;
}

pir_status pir_plan_launch(pir_plan *pl, pir_stream stream) {
  if (!pl) return PIR_ERR_INVALID_ARG;
  DeviceGuard g(pl->ctx->device);
  HIP_OR_FAIL(pl->ctx, hipGraphLaunch(pl->exec, (hipStream_t)stream));
  return PIR_OK;
}

void pir_plan_destroy(pir_plan *pl) {
  if (!pl) return;
  DeviceGuard g(pl->ctx->device);
  (void)hipDeviceSynchronize();
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  dev_free(pl->ctx, pl->ws, pl->ws_bytes);
  delete pl;
}

pir_status pir_tune_batch(pir_ctx *ctx, const pir_job *jobs, size_t n_jobs, pir_stream stream,
                          char *report, size_t report_len) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  if (!jobs || n_jobs == 0) return fail(ctx, PIR_ERR_INVALID_ARG, "no jobs");
  BatchPlan p;
  pir_status st = plan_batch(ctx, jobs, n_jobs, p);
  if (st != PIR_OK) return st;
  DeviceGuard g(ctx->device);
  if ((st = ensure_ws(ctx, p.bytes())) != PIR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  place_batch(jobs, n_jobs, (uint8_t *)ctx->ws, p);
  HIP_OR_FAIL(ctx, launch_fill_tuning((uint32_t *)ctx->ws, p.bytes() / 4, s));
  hipEvent_t e0, e1;
  HIP_OR_FAIL(ctx, hipEventCreate(&e0));
  HIP_OR_FAIL(ctx, hipEventCreate(&e1));
  std::string rep;
  for (const std::vector<ScanJob> *grp : {&p.b1, &p.mf}) {
    if (grp->empty()) continue;
    uint32_t bmax = 0;
    for (const ScanJob &j : *grp) bmax = std::max(bmax, j.B);
    const std::vector<ScanCfg> cands = scan_candidates(bmax);
    float best = 1e30f;
    size_t best_i = 0;
    for (size_t i = 0; i < cands.size(); ++i) {
      float ms = 0.f;
      HIP_OR_FAIL(ctx, time_launches([&] { return launch_scan(grp->data(), grp->size(), cands[i], s); },
                                     s, e0, e1, &ms));
      char buf[96];
      snprintf(buf, sizeof buf, "%s%zu:%u/%u/%u/%u=%.4f;", grp == &p.b1 ? "b1 " : "mf ", i,
               cands[i].kind, cands[i].jbw, cands[i].unr, cands[i].nt, ms);
      rep += buf;
      if (ms < best) best = ms, best_i = i;
    }
    ctx->batch_cfg[group_key(*grp)] = cands[best_i];
    char buf[32];
    snprintf(buf, sizeof buf, "best=%zu;", best_i);
    rep += buf;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (report && report_len) {
    std::strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return PIR_OK;
}

uint32_t pir_scan_variants(uint32_t B) {
  return (B >= 1 && B <= PIR_MAX_BATCH) ? (uint32_t)scan_candidates(B).size() : 0;
}

const char *pir_scan_kernel(const pir_ctx *ctx, const pir_db *db, uint32_t B) {
  if (!ctx || !db || B < 1 || B > PIR_MAX_BATCH) return nullptr;
  return scan_kernel_name(chosen_cfg(ctx, db->desc, B), db->desc);
}

pir_status pir_scan_select(pir_ctx *ctx, const pir_db *db, uint32_t B, uint32_t index) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  if (!db || B < 1 || B > PIR_MAX_BATCH) return fail(ctx, PIR_ERR_INVALID_ARG, "bad db or B");
  const std::vector<ScanCfg> c = scan_candidates(B);
  if (index >= c.size()) return fail(ctx, PIR_ERR_INVALID_ARG, "variant %u out of range", index);
  ctx->scan_cfg[shape_key(db->desc, B)] = c[index];
  return PIR_OK;
}

pir_status pir_tune(pir_ctx *ctx, const pir_db *db, uint32_t B, pir_stream stream, char *report,
                    size_t report_len) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  if (!db || B < 1 || B > PIR_MAX_BATCH) return fail(ctx, PIR_ERR_INVALID_ARG, "bad db or B");
  if (db->ctx != ctx) return fail(ctx, PIR_ERR_INVALID_ARG, "database belongs to another context");
  DeviceGuard g(ctx->device);
  const DbDesc &d = db->desc;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t qb = al((size_t)B * d.R * 2 * d.K * d.N * 4);
  const size_t ab = al(query_atom_bytes(d, B));
  const size_t ob = al((size_t)B * d.C * 2 * d.K * d.N * 4);
  pir_status st = ensure_ws(ctx, qb + ab + ob);
  if (st != PIR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  uint8_t *base = (uint8_t *)ctx->ws;
  // Time on random-looking operands: the matrix cores draw more power (and
  // clock lower) on them than on zeros, which can change the ranking.
  HIP_OR_FAIL(ctx, launch_fill_tuning((uint32_t *)base, (qb + ab + ob) / 4, s));
  ScanJob job{d, base + qb, (const uint32_t *)base, (uint32_t *)(base + qb + ab), B, 0, d.K * d.N, 0,
              0};
  const std::vector<ScanCfg> cands = scan_candidates(B);
  hipEvent_t e0, e1;
  HIP_OR_FAIL(ctx, hipEventCreate(&e0));
  HIP_OR_FAIL(ctx, hipEventCreate(&e1));
  std::string rep;
  float best = 1e30f;
  size_t best_i = 0;
  for (size_t i = 0; i < cands.size(); ++i) {
    float ms = 0.f;
    HIP_OR_FAIL(ctx, time_launches([&] { return launch_scan(&job, 1, cands[i], s); }, s, e0, e1, &ms));
    char buf[96];
    snprintf(buf, sizeof buf, "%zu:%u/%u/%u/%u=%.4f;", i, cands[i].kind, cands[i].jbw, cands[i].unr,
             cands[i].nt, ms);
    rep += buf;
    if (ms < best) best = ms, best_i = i;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->scan_cfg[shape_key(d, B)] = cands[best_i];
  char buf[32];
  snprintf(buf, sizeof buf, "best=%zu", best_i);
  rep += buf;
  if (report && report_len) {
    std::strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return PIR_OK;
}

pir_status pir_profile_stages(pir_ctx *ctx, uint32_t mask) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  if (mask >> PIR_N_STAGES) return fail(ctx, PIR_ERR_INVALID_ARG, "stage mask 0x%x", mask);
  DeviceGuard g(ctx->device);
  profile_drain(ctx);
  for (int i = 0; i < PIR_N_STAGES; ++i) ctx->stage_ms[i] = 0, ctx->stage_n[i] = 0;
  ctx->prof = mask;
  return PIR_OK;
}

pir_status pir_profile_enable(pir_ctx *ctx, int enable) {
  return pir_profile_stages(ctx, enable ? (1u << PIR_N_STAGES) - 1 : 0u);
}

pir_status pir_profile_read(pir_ctx *ctx, uint32_t stage, double *total_ms, uint64_t *launches) {
  if (!ctx || stage >= PIR_N_STAGES) return PIR_ERR_INVALID_ARG;
  DeviceGuard g(ctx->device);
  profile_drain(ctx);
  if (total_ms) *total_ms = ctx->stage_ms[stage];
  if (launches) *launches = ctx->stage_n[stage];
  return PIR_OK;
}

}  // extern "C"
