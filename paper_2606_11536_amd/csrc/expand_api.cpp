// Host side of query expansion (ExpPack, Sec. 3.5 and App. C.2) and RGSW
// folding (Sec. 3.2 step 7, Sec. 3.6): validation, workspace layout and the
// per-level launch sequence.  The kernels are in expand.hip; the transforms
// are the row NTTs of ntt.hip.
//
// Expansion level j (j = 0 .. l-1, l = ceil(log2 n)) of every client turns
// its P_in = min(2^j, n) ciphertexts into P_out = min(2^(j+1), n): output m
// comes from input k = m mod 2^j on branch m >> j (branch 1 multiplies by
// X^-(2^j) first) as c + Subs(c, N/2^j + 1), Subs = automorphism then key
// switch.  One level is five launches: digits of the automorphed mask, their
// NTT, the digit-key products, the inverse NTT, and the combine.  Outputs at
// or past n are never computed (their descendants all lie past n).
#include <algorithm>

#include "ctx.h"
#include "expand_internal.h"

using namespace pir;

struct pir_keys {
  pir_ctx *ctx = nullptr;
  pir_params params{};
  const DevPrime *primes = nullptr;
  uint32_t B = 0, levels = 0, base_log = 0, n_digits = 0;
  uint32_t *dev = nullptr;  // [B][levels][n_digits][2][K][N], NTT form
  size_t bytes = 0;
};

namespace {

uint64_t inv_mod(uint64_t a, uint64_t m) {
  int64_t r0 = (int64_t)m, r1 = (int64_t)(a % m), t0 = 0, t1 = 1;
  while (r1 != 0) {
    const int64_t qt = r0 / r1, r2 = r0 - qt * r1, t2 = t0 - qt * t1;
    r0 = r1, r1 = r2, t0 = t1, t1 = t2;
  }
  return (uint64_t)((t0 % (int64_t)m + (int64_t)m) % (int64_t)m);
}

uint64_t pow_mod(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = (unsigned __int128)r * b % m;
    b = (unsigned __int128)b * b % m;
    e >>= 1;
  }
  return r;
}

pir_status gadget_of(pir_ctx *ctx, const pir_params *p, uint32_t base_log, uint32_t n_digits,
                     GadgetArgs *g) {
  pir_status st = check_params(ctx, p);
  if (st != PIR_OK) return st;
  if (p->n_primes > 2)
    return fail(ctx, PIR_ERR_UNSUPPORTED, "expansion and folding take 1 or 2 primes, not %u",
                p->n_primes);
  if (base_log < 1 || base_log > 30 || n_digits < 1 || n_digits > PIR_MAX_DIGITS)
    return fail(ctx, PIR_ERR_INVALID_ARG, "base_log=%u or n_digits=%u out of range", base_log,
                n_digits);
  g->K = p->n_primes;
  g->q0 = p->primes[0];
  g->q1 = g->K == 2 ? p->primes[1] : 1;
  g->Q = (uint64_t)g->q0 * g->q1;
  g->c = g->K == 2 ? (double)inv_mod(g->q0, g->q1) : 0.0;
  g->inv_q0 = 1.0 / (double)g->q0;
  g->inv_q1 = 1.0 / (double)g->q1;
  g->base_log = base_log;
  g->n_digits = n_digits;
  const uint32_t bits = base_log * n_digits;
  if (bits < 64 && (1ull << bits) < g->Q)
    return fail(ctx, PIR_ERR_INVALID_ARG, "2^(base_log n_digits) = 2^%u does not cover Q", bits);
  return PIR_OK;
}

uint32_t levels_for(uint32_t n) {
  uint32_t l = 0;
  while ((1u << l) < n) ++l;
  return std::max(l, 1u);
}

}  // namespace

extern "C" {

pir_status pir_expand_keys_load(pir_ctx *ctx, const pir_params *params, const uint32_t *keys,
                                int keys_is_device, uint32_t B, uint32_t levels,
                                uint32_t base_log, uint32_t n_digits, pir_stream stream,
                                pir_keys **out) {
  if (!ctx || !out) return PIR_ERR_INVALID_ARG;
  *out = nullptr;
  GadgetArgs g{};
  pir_status st = gadget_of(ctx, params, base_log, n_digits, &g);
  if (st != PIR_OK) return st;
  if (!keys) return fail(ctx, PIR_ERR_INVALID_ARG, "keys is NULL");
  if (B < 1 || B > PIR_MAX_BATCH || levels < 1 || levels > params->log2_n)
    return fail(ctx, PIR_ERR_INVALID_ARG, "B=%u or levels=%u out of range", B, levels);
  DeviceGuard dg(ctx->device);
  const DevPrime *primes = nullptr;
  if ((st = prime_set(ctx, params, &primes)) != PIR_OK) return st;
  const size_t N = (size_t)1 << params->log2_n, K = params->n_primes;
  const size_t rows = (size_t)B * levels * n_digits * 2 * K;
  pir_keys *k = new (std::nothrow) pir_keys;
  if (!k) return fail(ctx, PIR_ERR_OUT_OF_MEMORY, "host allocation failed");
  k->ctx = ctx;
  k->params = *params;
  k->primes = primes;
  k->B = B;
  k->levels = levels;
  k->base_log = base_log;
  k->n_digits = n_digits;
  k->bytes = rows * N * 4;
  if ((st = dev_alloc(ctx, (void **)&k->dev, k->bytes, "expansion keys")) != PIR_OK) {
    delete k;
    return st;
  }
  hipStream_t s = (hipStream_t)stream;
  const hipError_t e = hipMemcpyAsync(k->dev, keys, k->bytes,
                                      keys_is_device ? hipMemcpyDeviceToDevice
                                                     : hipMemcpyHostToDevice, s);
  if (e != hipSuccess || launch_ntt(k->dev, rows, (uint32_t)K, params->log2_n, primes, false, s) !=
                             hipSuccess) {
    (void)hipStreamSynchronize(s);
    dev_free(ctx, k->dev, k->bytes);
    delete k;
    return fail(ctx, PIR_ERR_DEVICE, "copy or transform of the expansion keys failed");
  }
  if (!keys_is_device && hipStreamSynchronize(s) != hipSuccess) {
    dev_free(ctx, k->dev, k->bytes);
    delete k;
    return fail(ctx, PIR_ERR_DEVICE, "copy of the expansion keys failed");
  }
  *out = k;
  return PIR_OK;
}

void pir_expand_keys_free(pir_keys *keys) {
  if (!keys) return;
  DeviceGuard dg(keys->ctx->device);
  (void)hipDeviceSynchronize();
  dev_free(keys->ctx, keys->dev, keys->bytes);
  delete keys;
}

pir_status pir_expand(pir_ctx *ctx, const pir_keys *keys, const uint32_t *ct_coeff, uint32_t n,
                      uint32_t *out, pir_stream stream) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  if (!keys || !ct_coeff || !out) return fail(ctx, PIR_ERR_INVALID_ARG, "null argument");
  if (keys->ctx != ctx) return fail(ctx, PIR_ERR_INVALID_ARG, "keys belong to another context");
  const pir_params &p = keys->params;
  const uint32_t N = 1u << p.log2_n, K = p.n_primes, B = keys->B;
  if (n < 1 || n > N) return fail(ctx, PIR_ERR_INVALID_ARG, "n=%u not in [1, N]", n);
  const uint32_t l = levels_for(n);
  if (l > keys->levels)
    return fail(ctx, PIR_ERR_INVALID_ARG, "n=%u needs %u levels of keys, %u loaded", n, l,
                keys->levels);
  GadgetArgs g{};
  pir_status st = gadget_of(ctx, &p, keys->base_log, keys->n_digits, &g);
  if (st != PIR_OK) return st;
  DeviceGuard dg(ctx->device);
  // workspace: two level buffers (inputs of a level, outputs of a non-final
  // level), the digits and the key-switched products of the widest level
  const size_t KN = (size_t)K * N, ct_words = 2 * KN;
  const size_t half = std::min<size_t>((size_t)1 << (l - 1), n);
  const size_t lvl_words = (size_t)B * half * ct_words;
  const size_t dig_words = (size_t)B * n * keys->n_digits * KN;
  const size_t acc_words = (size_t)B * n * ct_words;
  const size_t ws_words = 2 * lvl_words + dig_words + acc_words;
  if ((st = ensure_ws(ctx, ws_words * 4)) != PIR_OK) return st;
  uint32_t *bufA = (uint32_t *)ctx->ws, *bufB = bufA + lvl_words;
  uint32_t *dig = bufB + lvl_words, *acc = dig + dig_words;
  hipStream_t s = (hipStream_t)stream;
  // level 0 input: the ciphertexts times 2^-l mod q_k
  HIP_OR_FAIL(ctx, hipMemcpyAsync(bufA, ct_coeff, (size_t)B * ct_words * 4,
                                  hipMemcpyDeviceToDevice, s));
  uint32_t f[2];
  for (uint32_t k = 0; k < K; ++k)
    f[k] = (uint32_t)inv_mod(pow_mod(2, l, p.primes[k]), p.primes[k]);
  HIP_OR_FAIL(ctx, launch_scale_rows(bufA, (size_t)B * 2 * K, p.log2_n, K, p.primes, f, s));
  const size_t key_stride = (size_t)keys->levels * keys->n_digits * ct_words;
  uint32_t *cur = bufA, *nxt = bufB;
  for (uint32_t j = 0; j < l; ++j) {
    const uint32_t p_in = std::min<uint32_t>(1u << j, n), p_out = std::min<uint32_t>(2u << j, n);
    const uint32_t gexp = N / (1u << j) + 1;
    const PolyMap m0{0, (uint32_t)inv_mod(gexp, 2ull * N)}, m1{1u << j, m0.g_inv};
    const uint32_t n_polys = B * p_out;
    uint32_t *dst = j + 1 == l ? out : nxt;
    HIP_OR_FAIL(ctx, launch_gadget_digits(cur, dig, n_polys, p_out, p_in, j, m0, m1, false,
                                          p.log2_n, g, s));
    HIP_OR_FAIL(ctx, launch_ntt(dig, (size_t)n_polys * keys->n_digits * K, K, p.log2_n,
                                keys->primes, false, s));
    HIP_OR_FAIL(ctx, launch_gadget_mac(dig, keys->dev + (size_t)j * keys->n_digits * ct_words,
                                       key_stride, p_out, acc, n_polys, keys->n_digits, p.log2_n,
                                       K, keys->primes, s));
    HIP_OR_FAIL(ctx, launch_ntt(acc, (size_t)n_polys * 2 * K, K, p.log2_n, keys->primes, true, s));
    HIP_OR_FAIL(ctx, launch_expand_combine(cur, acc, dst, CombineArgs{B, p_in, j, p_out}, m0, m1,
                                           p.log2_n, K, p.primes, s));
    std::swap(cur, nxt);
  }
  return PIR_OK;
}

pir_status pir_fold(pir_ctx *ctx, const pir_params *params, const uint32_t *cts_coeff, uint32_t D,
                    const uint32_t *rgsw_coeff, uint32_t base_log, uint32_t n_digits, uint32_t B,
                    uint32_t *out, pir_stream stream) {
  if (!ctx) return PIR_ERR_INVALID_ARG;
  GadgetArgs g{};
  pir_status st = gadget_of(ctx, params, base_log, n_digits, &g);
  if (st != PIR_OK) return st;
  if (!cts_coeff || !out || (D > 1 && !rgsw_coeff))
    return fail(ctx, PIR_ERR_INVALID_ARG, "null argument");
  if (B < 1 || B > PIR_MAX_BATCH || D < 1 || D > (1u << 20) || (D & (D - 1)))
    return fail(ctx, PIR_ERR_INVALID_ARG, "B=%u or D=%u (a power of two) out of range", B, D);
  uint32_t L = 0;
  while ((1u << L) < D) ++L;
  const uint32_t N = 1u << params->log2_n, K = params->n_primes;
  const size_t KN = (size_t)K * N, ct_words = 2 * KN;
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  if (L == 0) {
    HIP_OR_FAIL(ctx, hipMemcpyAsync(out, cts_coeff, (size_t)B * ct_words * 4,
                                    hipMemcpyDeviceToDevice, s));
    return PIR_OK;
  }
  const DevPrime *primes = nullptr;
  if ((st = prime_set(ctx, params, &primes)) != PIR_OK) return st;
  // workspace: the RGSW rows in NTT form, two level buffers, digits, products
  const size_t rgsw_words = (size_t)B * L * 2 * n_digits * ct_words;
  const size_t pairs0 = (size_t)B * (D / 2);
  const size_t lvl_words = pairs0 * ct_words;
  const size_t dig_words = pairs0 * 2 * n_digits * KN;
  const size_t ws_words = rgsw_words + 2 * lvl_words + dig_words + lvl_words;
  if ((st = ensure_ws(ctx, ws_words * 4)) != PIR_OK) return st;
  uint32_t *rg = (uint32_t *)ctx->ws, *bufA = rg + rgsw_words, *bufB = bufA + lvl_words;
  uint32_t *dig = bufB + lvl_words, *acc = dig + dig_words;
  HIP_OR_FAIL(ctx, hipMemcpyAsync(rg, rgsw_coeff, rgsw_words * 4, hipMemcpyDeviceToDevice, s));
  HIP_OR_FAIL(ctx, launch_ntt(rg, rgsw_words / N, K, params->log2_n, primes, false, s));
  const size_t rg_stride = (size_t)L * 2 * n_digits * ct_words;
  const uint32_t *cur = cts_coeff;
  uint32_t *nxt = bufA, *other = bufB;
  for (uint32_t j = 0; j < L; ++j) {
    const uint32_t pairs = D >> (j + 1);
    const uint32_t n_polys = B * pairs;
    uint32_t *dst = j + 1 == L ? out : nxt;
    HIP_OR_FAIL(ctx, launch_gadget_digits(cur, dig, n_polys, 0, 0, 0, PolyMap{0, 1},
                                          PolyMap{0, 1}, true, params->log2_n, g, s));
    HIP_OR_FAIL(ctx, launch_ntt(dig, (size_t)n_polys * 2 * n_digits * K, K, params->log2_n,
                                primes, false, s));
    HIP_OR_FAIL(ctx, launch_gadget_mac(dig, rg + (size_t)j * 2 * n_digits * ct_words, rg_stride,
                                       pairs, acc, n_polys, 2 * n_digits, params->log2_n, K, primes,
                                       s));
    HIP_OR_FAIL(ctx, launch_ntt(acc, (size_t)n_polys * 2 * K, K, params->log2_n, primes, true, s));
    HIP_OR_FAIL(ctx, launch_fold_combine(cur, acc, dst, n_polys, params->log2_n, K,
                                         params->primes, s));
    cur = dst;
    std::swap(nxt, other);
  }
  return PIR_OK;
}

}  // extern "C"
