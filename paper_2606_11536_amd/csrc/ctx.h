// Host-side internals of libpir shared by the C ABI implementation files:
// the context and database objects, error reporting, device allocation under
// the context's HBM budget.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <string>
#include <vector>

#include "pir_internal.h"

struct pir_ctx {
  int device = 0;
  int num_cus = 0;
  size_t budget = 0;  // 0 = unlimited
  size_t held = 0;    // device bytes held (databases + workspace + tables)
  std::string err;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  // device address of the library's fixed scratch array on this device
  // (pir_answer_batch_static), or null with the reason
  void *scratch = nullptr;
  std::string scratch_err;
  std::map<std::pair<uint32_t, uint32_t>, uint32_t *> tw_tables;  // (log2n, q) -> [4][N]
  std::map<std::vector<uint32_t>, pir::DevPrime *> prime_sets;       // (log2n, q...) -> [K]
  // stage profiling
  uint32_t prof = 0;  // bit (1 << stage) set: that stage is timed
  struct Rec {
    uint32_t stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  double stage_ms[PIR_N_STAGES] = {};
  uint64_t stage_n[PIR_N_STAGES] = {};
  // chosen scan variant per (N, K, R, C, B), and per fused job list
  std::map<std::array<uint32_t, 5>, pir::ScanCfg> scan_cfg;
  std::map<std::vector<uint32_t>, pir::ScanCfg> batch_cfg;
};

// A scalar-HE database: D1 x D0 int8 entries in GEMM atoms.
struct pir_sdb {
  pir_ctx *ctx = nullptr;
  uint32_t D1 = 0, D0 = 0, n_rb = 0, n_kb = 0;
  size_t bytes = 0;
  uint8_t *atoms = nullptr;
};

struct pir_db {
  pir_ctx *ctx = nullptr;
  pir_params params{};
  uint32_t R = 0, C = 0;
  uint32_t pack_d1 = 0;  // ring-packing hint: rows D1 of the LWE matrix (0: a database)
  size_t bytes = 0;
  uint8_t *atoms = nullptr;
  pir::DbDesc desc{};
};

namespace pir {

// Record an error message on ctx (or, without a context, for this thread) and
// return s.
pir_status fail(pir_ctx *ctx, pir_status s, const char *fmt, ...);
pir_status dev_alloc(pir_ctx *ctx, void **p, size_t bytes, const char *what);
void dev_free(pir_ctx *ctx, void *p, size_t bytes);
// The context workspace grown to at least `bytes` (synchronizes the device
// when it grows).
pir_status ensure_ws(pir_ctx *ctx, size_t bytes);
// Validation of ring parameters (UNSUPPORTED / INVALID_ARG with a message).
pir_status check_params(pir_ctx *ctx, const pir_params *p);
// Device constants for (log2n, primes), cached on the context.
pir_status prime_set(pir_ctx *ctx, const pir_params *p, const DevPrime **out);
// The chosen scan variant for (db shape, B).
ScanCfg chosen_cfg(const pir_ctx *ctx, const DbDesc &d, uint32_t B);
// The batched-kernel variant the server uses for (db shape, B): the tuned one
// if pir_tune chose a batched variant for this shape, else the default.
inline ScanCfg server_scan_cfg(const pir_ctx *ctx, const DbDesc &d, uint32_t B) {
  const ScanCfg c = chosen_cfg(ctx, d, B);
  return c.kind == 1 ? c : scan_default_mfma(B);
}

#define HIP_OR_FAIL(ctx, expr)                                                           \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail((ctx), PIR_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace pir
