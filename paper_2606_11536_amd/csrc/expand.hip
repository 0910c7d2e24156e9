// Query expansion and RGSW folding on the GPU (paper: ExpPack, Sec. 3.5 and
// App. C.2; poly-HE folding by RGSW-RLWE external products, Sec. 3.2 step 7
// and Sec. 3.6).
//
// Both are built from one step: take the balanced gadget digits of a
// polynomial (coefficient form), transform the digits to NTT form, and sum
// their slot-wise products with the rows of a key (key switching) or of an
// RGSW ciphertext.  The kernels here do the coefficient-form parts:
//  * k_gadget_digits: a signed permutation of the coefficients (a monomial
//    product X^-shift, then the automorphism X -> X^g) or a difference of two
//    ciphertexts, the CRT of the two residues into [0, Q), centring, and the
//    digits, written as residues ready for the row NTT;
//  * k_gadget_mac: the slot-wise digit-row products (NTT form);
//  * k_expand_combine / k_fold_combine: the sums that finish an expansion
//    level (c + Subs(c)) or a CMux (ct0 + RGSW [x] (ct1 - ct0)).
// Every value is an exact integer: CRT values are below Q = q0 q1 < 2^56 and
// are held in 64-bit integers; residue products go through the exact fp64
// product below.
#include "expand_internal.h"

namespace pir {
namespace {

constexpr int kThreads = 256;

// y * w mod q for exact integers |y| < 2^53, 0 <= w < q < 2^28: p = y w
// rounded, e = fma(y, w, -p) its exact error, r = fma(-rint(p/q), q, p) + e,
// exact with |r| < 0.51 q.
__device__ __forceinline__ double mulmod_exact(double y, double w, double q, double inv_q) {
  const double p = y * w;
  const double e = __builtin_fma(y, w, -p);
  return __builtin_fma(-__builtin_rint(p * inv_q), q, p) + e;
}

__device__ __forceinline__ uint32_t canon_f64(double r, double q, double inv_q) {
  const double t = __builtin_fma(-__builtin_rint(r * inv_q), q, r);  // |t| < 0.51 q
  return (uint32_t)(int)(t < 0.0 ? t + q : t);
}

// Source coefficient of output position pos of map(c), and whether it is
// negated: map = automorphism(g) after the product by X^-shift.
__device__ __forceinline__ uint32_t map_src(uint32_t pos, const PolyMap &m, uint32_t N,
                                            bool &neg) {
  const uint32_t j0 = (uint32_t)(((uint64_t)pos * m.g_inv) & (2 * N - 1));
  bool n1 = j0 >= N;
  const uint32_t j1 = n1 ? j0 - N : j0;
  const uint32_t i = j1 + m.shift;
  const bool n2 = i >= N;
  neg = n1 != n2;
  return n2 ? i - N : i;
}

// The centred CRT value of residues (x0, x1) (x1 ignored for K = 1).
__device__ __forceinline__ int64_t crt_centred(uint32_t x0, uint32_t x1, const GadgetArgs &g) {
  uint64_t x = x0;
  if (g.K == 2) {
    const double q1 = (double)g.q1;
    const double r = mulmod_exact((double)x1 - (double)x0, g.c, q1, g.inv_q1);  // |r| < 0.51 q1
    const uint32_t y = (uint32_t)(int)(r < 0.0 ? r + q1 : r);
    x += (uint64_t)g.q0 * y;                                                  // < Q
  }
  return x > g.Q / 2 ? (int64_t)x - (int64_t)g.Q : (int64_t)x;
}

// Writes the n_digits digits of x (|x| <= (Q-1)/2) at out[d * stride] as
// residues mod q_k (K rows of N words apart).  A digit can exceed a small
// prime (lower digits reach 2^(base_log-1), up to 2^29; the top digit takes
// the rest, below 2^29 because the gadget covers Q < 2^56 with base_log <= 30),
// so each is reduced exactly: it is an integer below 2^53, exact as a double.
__device__ __forceinline__ void put_digits(int64_t x, uint32_t *out, size_t dstride,
                                           uint32_t N, const GadgetArgs &g) {
  const int64_t B = (int64_t)1 << g.base_log, half = B >> 1;
  for (uint32_t d = 0; d < g.n_digits; ++d) {
    int64_t r = x;
    if (d + 1 < g.n_digits) {
      r = x & (B - 1);
      if (r >= half) r -= B;
      x = (x - r) >> g.base_log;
    }
    out[d * dstride] = canon_f64((double)r, (double)g.q0, g.inv_q0);
    if (g.K == 2) out[d * dstride + N] = canon_f64((double)r, (double)g.q1, g.inv_q1);
  }
}

// One thread per coefficient position of one polynomial (grid: N / 256 x polys).
__global__ __launch_bounds__(kThreads) void k_gadget_digits(const uint32_t *__restrict__ src,
                                                            uint32_t *__restrict__ dig,
                                                            uint32_t p_out, uint32_t p_in,
                                                            uint32_t level_bit, PolyMap m0,
                                                            PolyMap m1, uint32_t diff,
                                                            uint32_t log2n, const GadgetArgs g) {
  const uint32_t N = 1u << log2n, KN = g.K * N;
  const uint32_t pos = blockIdx.x * kThreads + threadIdx.x;
  const size_t p = blockIdx.y;
  uint32_t x0, x1 = 0;
  int64_t x;
  if (diff) {
    // digits of src[2p + 1] - src[2p], both components: dig[p][2 n_digits][K][N]
    const uint32_t *c0 = src + 2 * p * 2 * KN, *c1 = c0 + 2 * KN;
    for (uint32_t comp = 0; comp < 2; ++comp) {
      x0 = c1[comp * KN + pos] + (g.q0 - c0[comp * KN + pos]);
      x0 = x0 >= g.q0 ? x0 - g.q0 : x0;
      if (g.K == 2) {
        x1 = c1[comp * KN + N + pos] + (g.q1 - c0[comp * KN + N + pos]);
        x1 = x1 >= g.q1 ? x1 - g.q1 : x1;
      }
      x = crt_centred(x0, x1, g);
      put_digits(x, dig + (p * 2 + comp) * g.n_digits * KN + pos, KN, N, g);
    }
    return;
  }
  // expansion: output m of this client is branch br = m >> level_bit of input k
  const size_t client = p / p_out;
  const uint32_t m = (uint32_t)(p % p_out);
  const uint32_t k = m & ((1u << level_bit) - 1), br = m >> level_bit;
  const uint32_t *c = src + (client * p_in + k) * 2 * KN;  // component 0
  bool neg;
  const uint32_t i = map_src(pos, br ? m1 : m0, N, neg);
  x0 = c[i];
  if (g.K == 2) x1 = c[N + i];
  x = crt_centred(x0, x1, g);
  put_digits(neg ? -x : x, dig + p * g.n_digits * KN + pos, KN, N, g);
}

// One thread per (poly, prime, slot); rows digit rows per poly.
__global__ __launch_bounds__(kThreads) void k_gadget_mac(const uint32_t *__restrict__ dig,
                                                         const uint32_t *__restrict__ keys,
                                                         size_t key_stride, uint32_t ppk,
                                                         uint32_t *__restrict__ acc,
                                                         uint32_t rows, uint32_t log2n,
                                                         uint32_t K,
                                                         const DevPrime *__restrict__ primes) {
  const uint32_t N = 1u << log2n, KN = K * N;
  const uint32_t kt = blockIdx.x * kThreads + threadIdx.x;  // k N + t
  if (kt >= KN) return;
  const size_t p = blockIdx.y;
  const uint32_t k = kt >> log2n;
  const double q = (double)primes[k].q, inv_q = 1.0 / q;
  const uint32_t *key = keys + (p / ppk) * key_stride + kt;
  const uint32_t *d = dig + p * rows * KN + kt;
  double s0 = 0.0, s1 = 0.0;  // |s| < rows * 0.51 q < 2^34: exact
  // unrolled so that several rows' loads are in flight at once
#pragma unroll 4
  for (uint32_t r = 0; r < rows; ++r) {
    const double dv = (double)d[(size_t)r * KN];
    s0 += mulmod_exact(dv, (double)key[(size_t)(2 * r) * KN], q, inv_q);
    s1 += mulmod_exact(dv, (double)key[(size_t)(2 * r + 1) * KN], q, inv_q);
  }
  uint32_t *o = acc + p * 2 * KN + kt;
  o[0] = canon_f64(s0, q, inv_q);
  o[KN] = canon_f64(s1, q, inv_q);
}

// One thread per (output poly, prime, coefficient).
__global__ __launch_bounds__(kThreads) void k_expand_combine(const uint32_t *__restrict__ src,
                                                             const uint32_t *__restrict__ ks,
                                                             uint32_t *__restrict__ out,
                                                             const CombineArgs a, PolyMap m0,
                                                             PolyMap m1, uint32_t log2n,
                                                             uint32_t K, uint32_t q0,
                                                             uint32_t q1) {
  const uint32_t N = 1u << log2n, KN = K * N;
  const uint32_t kt = blockIdx.x * kThreads + threadIdx.x;
  if (kt >= KN) return;
  const size_t p = blockIdx.y;  // client * out_per_client + m
  const size_t client = p / a.out_per_client;
  const uint32_t m = (uint32_t)(p % a.out_per_client);
  const uint32_t k = m & ((1u << a.level_bit) - 1), br = m >> a.level_bit;
  const uint32_t kk = kt >> log2n, pos = kt & (N - 1);
  const uint32_t q = kk == 0 ? q0 : q1;
  const uint32_t *c = src + (client * a.P_in + k) * 2 * KN + kk * N;
  const PolyMap &mp = br ? m1 : m0;
  // the branch polynomial h = c X^-shift at pos, both components
  const PolyMap shift_only{mp.shift, 1};
  bool neg;
  uint32_t i = map_src(pos, shift_only, N, neg);
  uint32_t h0 = c[i], h1 = c[KN + i];
  if (neg) h0 = h0 ? q - h0 : 0, h1 = h1 ? q - h1 : 0;
  // tau(h_1) at pos
  i = map_src(pos, mp, N, neg);
  uint32_t t1 = c[KN + i];
  if (neg) t1 = t1 ? q - t1 : 0;
  const uint32_t *r = ks + p * 2 * KN + kt;
  uint32_t o0 = h0 + r[0];                 // < 2q < 2^29
  uint32_t o1 = h1 + t1;                   // < 2q
  o0 = o0 >= q ? o0 - q : o0;
  o1 = o1 >= q ? o1 - q : o1;
  o1 += r[KN];
  o1 = o1 >= q ? o1 - q : o1;
  uint32_t *o = out + p * 2 * KN + kt;
  o[0] = o0;
  o[KN] = o1;
}

__global__ __launch_bounds__(kThreads) void k_fold_combine(const uint32_t *__restrict__ src,
                                                           const uint32_t *__restrict__ ext,
                                                           uint32_t *__restrict__ out,
                                                           uint32_t log2n, uint32_t K,
                                                           uint32_t q0, uint32_t q1) {
  const uint32_t N = 1u << log2n, W = 2 * K * N;
  const uint32_t w = blockIdx.x * kThreads + threadIdx.x;  // (comp, k, t)
  if (w >= W) return;
  const size_t p = blockIdx.y;
  const uint32_t q = ((w >> log2n) % K) == 0 ? q0 : q1;
  const uint32_t v = src[2 * p * W + w] + ext[p * W + w];
  out[p * W + w] = v >= q ? v - q : v;
}

__global__ __launch_bounds__(kThreads) void k_scale_rows(uint32_t *__restrict__ x, uint32_t log2n,
                                                         uint32_t K, uint32_t q0, uint32_t q1,
                                                         uint32_t f0, uint32_t f1) {
  const size_t row = blockIdx.y;
  const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= (1u << log2n)) return;
  const bool first = row % K == 0;
  const double q = (double)(first ? q0 : q1), f = (double)(first ? f0 : f1);
  uint32_t *p = x + (row << log2n) + t;
  *p = canon_f64(mulmod_exact((double)*p, f, q, 1.0 / q), q, 1.0 / q);
}

dim3 grid_for(uint32_t words, size_t polys) {
  return dim3((words + kThreads - 1) / kThreads, (unsigned)polys);
}

}  // namespace

hipError_t launch_gadget_digits(const uint32_t *src, uint32_t *dig, uint32_t n_polys,
                                uint32_t p_out, uint32_t p_in, uint32_t level_bit, PolyMap m0,
                                PolyMap m1, bool diff, uint32_t log2n, const GadgetArgs &g,
                                hipStream_t s) {
  if (n_polys == 0) return hipSuccess;
  if (log2n < 8 || (g.K != 1 && g.K != 2) || (!diff && p_out == 0)) return hipErrorInvalidValue;
  k_gadget_digits<<<grid_for(1u << log2n, n_polys), kThreads, 0, s>>>(
      src, dig, p_out, p_in, level_bit, m0, m1, diff ? 1u : 0u, log2n, g);
  return hipGetLastError();
}

hipError_t launch_gadget_mac(const uint32_t *dig, const uint32_t *keys, size_t key_stride,
                             uint32_t polys_per_key, uint32_t *acc, uint32_t n_polys,
                             uint32_t rows, uint32_t log2n, uint32_t K, const DevPrime *primes,
                             hipStream_t s) {
  if (n_polys == 0) return hipSuccess;
  if (polys_per_key == 0 || rows == 0) return hipErrorInvalidValue;
  k_gadget_mac<<<grid_for(K << log2n, n_polys), kThreads, 0, s>>>(dig, keys, key_stride,
                                                                  polys_per_key, acc, rows, log2n,
                                                                  K, primes);
  return hipGetLastError();
}

hipError_t launch_expand_combine(const uint32_t *src, const uint32_t *ks, uint32_t *out,
                                 const CombineArgs &a, PolyMap m0, PolyMap m1, uint32_t log2n,
                                 uint32_t K, const uint32_t *q, hipStream_t s) {
  const size_t n = (size_t)a.B * a.out_per_client;
  if (n == 0) return hipSuccess;
  k_expand_combine<<<grid_for(K << log2n, n), kThreads, 0, s>>>(src, ks, out, a, m0, m1, log2n,
                                                               K, q[0], K == 2 ? q[1] : 1);
  return hipGetLastError();
}

hipError_t launch_fold_combine(const uint32_t *src, const uint32_t *ext, uint32_t *out,
                               uint32_t n_polys, uint32_t log2n, uint32_t K, const uint32_t *q,
                               hipStream_t s) {
  if (n_polys == 0) return hipSuccess;
  k_fold_combine<<<grid_for(2 * K << log2n, n_polys), kThreads, 0, s>>>(src, ext, out, log2n, K,
                                                                       q[0], K == 2 ? q[1] : 1);
  return hipGetLastError();
}

hipError_t launch_scale_rows(uint32_t *x, size_t n_rows, uint32_t log2n, uint32_t K,
                             const uint32_t *q, const uint32_t *f, hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  k_scale_rows<<<grid_for(1u << log2n, n_rows), kThreads, 0, s>>>(
      x, log2n, K, q[0], K == 2 ? q[1] : 1, f[0], K == 2 ? f[1] : 0);
  return hipGetLastError();
}

}  // namespace pir
