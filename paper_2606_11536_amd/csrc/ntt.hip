// Negacyclic NTT / INTT over Z_q[X]/(X^N + 1), q < 2^28, N in {1024, 2048, 4096}
// (paper: Sec. 2.3; single-kernel transform of Sec. 4.3).
//
// One workgroup transforms one residue row of N values: 256 threads for
// N <= 2048, 512 for N = 4096 (so that a thread holds at most 8 values and
// stays near 60 VGPRs, eight waves per SIMD).  Each thread keeps E values in
// registers and performs log2(E) radix-2 stages on them before the block
// exchanges values through LDS; the log2(N) stages therefore take
// ceil(log2 N / log2 E) register rounds.
//
// Forward: Cooley-Tukey stages with half-sizes N/2, N/4, ..., 1; the stage
// with half-size h uses twiddle psi^brv(N/(2h) + x/(2h)) for the pair
// (x, x + h).  Natural-order input, output slot t = a(psi^(2 brv(t) + 1)).
// Inverse: Gentleman-Sande stages with half-sizes 1, 2, ..., N/2 and the
// inverse twiddles, then the factor N^-1.
//
// Arithmetic: exact integers held in fp64 (full-rate FMA, where 32-bit
// integer multiplies run at quarter rate).  The product y*w mod q is
//   p = y*w (rounded), e = fma(y, w, -p)  (so y*w = p + e exactly),
//   r = fma(-rint(p/q), q, p) + e,
// exact because p - rint(p/q) q is an integer of magnitude below q/2 + q/1024
// and e is at most half an ulp of p; |r| < 0.51 q.  Values are not reduced
// between stages: forward stages add at most 0.51 q per stage (|x| < 8q),
// inverse stages at most double (|x| < 2^12 q < 2^41), so every product
// stays below 2^70 and every sum is an exact integer below 2^53.  Each value
// is reduced to [0, q) once at the end.
#include <cmath>

#include "device_util.h"
#include "pir_internal.h"

namespace pir {
namespace {

template <int LOGN>
struct Geo {
  static constexpr int N = 1 << LOGN;
  static constexpr int LT = LOGN >= 12 ? 9 : 8;  // log2 of threads per row
  static constexpr int T = 1 << LT;
  static constexpr int LE = LOGN - LT;  // log2 of values per thread
  static constexpr int E = 1 << LE;
  static constexpr int ROUNDS = (LOGN + LE - 1) / LE;
  static constexpr int REM = LOGN - (ROUNDS - 1) * LE;  // stages in the short round

  // stages done in round r
  static constexpr int s(int r, bool inv) {
    return inv ? (r == 0 ? REM : LE) : ((LOGN - r * LE) < LE ? (LOGN - r * LE) : LE);
  }
  // log2 of the smallest half-size in round r
  static constexpr int logL(int r, bool inv) {
    return inv ? (r == 0 ? 0 : REM + (r - 1) * LE) : (LOGN - 1 - r * LE) - (s(r, inv) - 1);
  }
};

// y * w mod q as an exact integer of magnitude below 0.51 q (see above).
__device__ __forceinline__ double mulmod_f64(double y, double w, double q, double inv_q) {
  const double p = y * w;
  const double e = __builtin_fma(y, w, -p);
  return __builtin_fma(-__builtin_rint(p * inv_q), q, p) + e;
}

// An exact integer v (|v| < 2^53) reduced to [0, q).
__device__ __forceinline__ uint32_t reduce_f64(double v, double q, double inv_q) {
  const double r = __builtin_fma(-__builtin_rint(v * inv_q), q, v);  // |r| < 0.51 q
  return (uint32_t)(int)(r < 0.0 ? r + q : r);
}

// Index of register e in round r for thread tid.
template <int LOGN, bool INV, int R>
__device__ __forceinline__ uint32_t ridx(uint32_t tid, int e) {
  using G = Geo<LOGN>;
  constexpr int S = G::s(R, INV);
  constexpr int LL = G::logL(R, INV);
  const uint32_t g = (uint32_t)e >> S;
  const uint32_t ep = (uint32_t)e & ((1u << S) - 1);
  const uint32_t gid = tid + g * G::T;
  const uint32_t x0 = ((gid >> LL) << (LL + S)) + (gid & ((1u << LL) - 1));
  return x0 + (ep << LL);
}

template <int LOGN, bool INV, int R>
__device__ __forceinline__ void round_compute(double (&x)[Geo<LOGN>::E], uint32_t tid,
                                              const uint32_t *__restrict__ tw, double q,
                                              double inv_q) {
  using G = Geo<LOGN>;
  constexpr int S = G::s(R, INV);
  constexpr int LL = G::logL(R, INV);
#pragma unroll
  for (int step = 0; step < S; ++step) {
    const int u = INV ? step : (S - 1 - step);
    const int logh = LL + u;
#pragma unroll
    for (int e = 0; e < G::E; ++e) {
      if ((e >> u) & 1) continue;
      const int f = e + (1 << u);
      const uint32_t idx = ridx<LOGN, INV, R>(tid, e);
      const uint32_t ti = (uint32_t)(G::N + idx) >> (logh + 1);
      // a global (not flat) load: the table pointer comes from the prime
      // record, so the compiler cannot tell its address space by itself
      const double w = (double)((const __attribute__((address_space(1))) uint32_t *)tw)[ti];
      const double X = x[e], Y = x[f];
      if (!INV) {
        const double T = mulmod_f64(Y, w, q, inv_q);
        x[e] = X + T;
        x[f] = X - T;
      } else {
        x[e] = X + Y;
        x[f] = mulmod_f64(X - Y, w, q, inv_q);
      }
    }
  }
}

template <int LOGN, bool INV, int R>
__device__ __forceinline__ void rounds_from(double (&x)[Geo<LOGN>::E], uint32_t tid, double *sm,
                                            const uint32_t *tw, double q, double inv_q) {
  using G = Geo<LOGN>;
  round_compute<LOGN, INV, R>(x, tid, tw, q, inv_q);
  if constexpr (R + 1 < G::ROUNDS) {
    if (R > 0) __syncthreads();  // the previous round's reads are done
#pragma unroll
    for (int e = 0; e < G::E; ++e) sm[ridx<LOGN, INV, R>(tid, e)] = x[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = sm[ridx<LOGN, INV, R + 1>(tid, e)];
    rounds_from<LOGN, INV, R + 1>(x, tid, sm, tw, q, inv_q);
  }
}

// Transform x (exact integers, loaded with round-0 indexing); on return out
// holds canonical residues in [0, q) laid out with last-round indexing.  The
// inverse multiplies by N^-1; a forward transform with scale != 0 multiplies
// every output by scale (mod q), which by linearity is the transform of the
// scaled input.  Inputs may be any integers of magnitude below 2^33 (forward)
// or 2^29 (inverse): the stage bounds above then still hold.
template <int LOGN, bool INV>
__device__ __forceinline__ void transform(double (&x)[Geo<LOGN>::E],
                                          uint32_t (&out)[Geo<LOGN>::E], uint32_t tid,
                                          double *sm, const DevPrime &P, uint32_t scale = 0) {
  constexpr int N = Geo<LOGN>::N;
  const double q = (double)P.q, inv_q = 1.0 / q;
  const uint32_t *tw = P.tw + (INV ? 2 * N : 0);
  rounds_from<LOGN, INV, 0>(x, tid, sm, tw, q, inv_q);
  const double f = INV ? (double)P.ninv : (double)scale;
  const bool mul = INV || scale != 0;
#pragma unroll
  for (int e = 0; e < Geo<LOGN>::E; ++e)
    out[e] = reduce_f64(mul ? mulmod_f64(x[e], f, q, inv_q) : x[e], q, inv_q);
}

// One residue row per block.  With an addend (inverse only): the rows are
// answer ciphertexts [..][2][K][N], and every row of a component-1 polynomial
// (p = row / K odd) first gets row (p / 2) K + row % K of `add` added -- the
// (0 | G) term of ring packing, added before the inverse transform (which is
// linear), so that no separate pass over the answers is needed.
template <int LOGN, bool INV, bool ADD>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_ntt_rows(const uint32_t *__restrict__ src,
                                                       uint32_t *__restrict__ dst, uint32_t K,
                                                       const DevPrime *__restrict__ primes,
                                                       const uint32_t *__restrict__ add) {
  using G = Geo<LOGN>;
  __shared__ double sm[G::N];
  const uint32_t tid = threadIdx.x;
  const size_t row = blockIdx.x;
  const DevPrime &P = primes[row % K];
  const uint32_t *in = src + row * G::N;
  uint32_t *out = dst + row * G::N;
  double x[G::E];
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = (double)in[ridx<LOGN, INV, 0>(tid, e)];
  if constexpr (ADD) {
    const size_t p = row / K;
    if (p & 1) {
      const uint32_t *a = add + ((p >> 1) * K + row % K) * G::N;
#pragma unroll
      for (int e = 0; e < G::E; ++e) x[e] += (double)a[ridx<LOGN, INV, 0>(tid, e)];
    }
  }
  uint32_t y[G::E];
  transform<LOGN, INV>(x, y, tid, sm, P);
  constexpr int LAST = G::ROUNDS - 1;
#pragma unroll
  for (int e = 0; e < G::E; ++e) out[ridx<LOGN, INV, LAST>(tid, e)] = y[e];
}

// raw: [rows][N] uint8 or uint32 (rows = S*C of the slab); out: [K][rows][N].
// The unsigned lift: a coefficient v < 2^32 is the integer v, reduced mod q_k
// by the transform's final reduction.
template <int LOGN, typename T>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_lift_ntt(const T *__restrict__ raw,
                                                       uint32_t *__restrict__ out, uint32_t rows,
                                                       uint32_t valid_rows,
                                                       const DevPrime *__restrict__ primes) {
  using G = Geo<LOGN>;
  __shared__ double sm[G::N];
  const uint32_t tid = threadIdx.x;
  const uint32_t row = blockIdx.x;
  const uint32_t k = blockIdx.y;
  const DevPrime &P = primes[k];
  double x[G::E];
  if (row < valid_rows) {
    const T *in = raw + (size_t)row * G::N;
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = (double)in[ridx<LOGN, false, 0>(tid, e)];
  } else {
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = 0.0;
  }
  uint32_t y[G::E];
  transform<LOGN, false>(x, y, tid, sm, P);
  uint32_t *o = out + ((size_t)k * rows + row) * G::N;
  constexpr int LAST = G::ROUNDS - 1;
#pragma unroll
  for (int e = 0; e < G::E; ++e) o[ridx<LOGN, false, LAST>(tid, e)] = y[e];
}

// The (0 | G) term of ring packing: G = NTT(Delta iota(b)) for every client
// beta and chunk r of its offsets b[beta][0 .. D1).  Row (beta, r), prime k:
// coefficient j is b[beta][r N + j] (zero past D1), lifted unsigned; by
// linearity the transform's output is scaled by Delta mod q_k (delta[k]).
// out: [B][C'][K][N].
struct OffsetArgs {
  uint32_t D1, Cp, K;
  uint32_t delta[PIR_MAX_PRIMES];
};

template <int LOGN>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_offset_ntt(const uint32_t *__restrict__ b,
                                                         uint32_t *__restrict__ out,
                                                         const DevPrime *__restrict__ primes,
                                                         const OffsetArgs a) {
  using G = Geo<LOGN>;
  __shared__ double sm[G::N];
  const uint32_t tid = threadIdx.x;
  const uint32_t row = blockIdx.x, k = blockIdx.y;
  const uint32_t beta = row / a.Cp, r = row % a.Cp;
  const uint32_t *in = b + (size_t)beta * a.D1;
  double x[G::E];
#pragma unroll
  for (int e = 0; e < G::E; ++e) {
    const uint32_t j = r * G::N + ridx<LOGN, false, 0>(tid, e);
    x[e] = j < a.D1 ? (double)in[j] : 0.0;
  }
  uint32_t y[G::E];
  transform<LOGN, false>(x, y, tid, sm, primes[k], a.delta[k]);
  uint32_t *o = out + ((size_t)row * a.K + k) * G::N;
  constexpr int LAST = G::ROUNDS - 1;
#pragma unroll
  for (int e = 0; e < G::E; ++e) o[ridx<LOGN, false, LAST>(tid, e)] = y[e];
}

// Modulus switching (Sec. 4.3 fuses it with the inverse NTT; App. D.5): the
// coefficient x in [0, Q) with residues x0 mod q0 (and x1 mod q1) becomes the
// nearest integer to x 2^bits / Q, reduced mod 2^bits.
//  * CRT (Garner): y = (x1 - x0) q0^-1 mod q1, x = x0 + q0 y < Q < 2^56.  The
//    signed difference x1 - x0 (|x1 - x0| < 2^28, whatever the sizes of q0
//    and q1) goes straight into the exact fp64 product of mulmod_f64, which
//    reduces any integer operand below 2^53 to within 0.51 q1 of zero;
//  * k = rint(x * (2^bits / Q)) in fp64 is within one of the nearest integer:
//    its error is below 2^-19 on a value below 2^32;
//  * the residual r = x 2^bits - k Q is computed in wrapping 64-bit integer
//    arithmetic, exact because |r| < 2 Q < 2^58; k moves by one when |2r| > Q.
//    2r = +-Q would be a tie, impossible for odd Q.
struct MsArgs {
  uint64_t Q;          // q0 q1 (q0 for one prime)
  double scale;        // 2^bits / Q
  double q1d, inv_q1;  // q1 and 1 / q1
  double c;            // q0^-1 mod q1
  uint32_t q0, q1, bits, mask;
};

template <bool TWO>
__device__ __forceinline__ uint32_t mod_switch(uint32_t x0, uint32_t x1, const MsArgs &m) {
  uint64_t x = x0;
  if constexpr (TWO) {
    const double d = (double)x1 - (double)x0;                      // |d| < 2^28
    const double r = mulmod_f64(d, m.c, m.q1d, m.inv_q1);          // |r| < 0.51 q1
    const uint32_t y = (uint32_t)(int)(r < 0.0 ? r + m.q1d : r);
    x += (uint64_t)m.q0 * y;
  }
  int64_t k = (int64_t)__builtin_rint((double)x * m.scale);
  const int64_t r = (int64_t)((x << m.bits) - (uint64_t)k * m.Q);
  const int64_t Q = (int64_t)m.Q;
  if (2 * r > Q) ++k;
  else if (2 * r < -Q) --k;
  return (uint32_t)k & m.mask;
}

// One block per answer polynomial [K][N] (K = 1 or 2): both residue rows are
// loaded up front, inverse-transformed one after the other in the same LDS,
// and every coefficient is switched on its way out: [N] words, no
// intermediate coefficient form in HBM.
// With an addend, odd polynomials (component 1 of [..][2] answers) first get
// polynomial poly / 2 of `add` ([..][K][N]) added, as in k_ntt_rows.
template <int LOGN, bool TWO, bool ADD>
__global__ __launch_bounds__(Geo<LOGN>::T) void k_intt_switch(const uint32_t *__restrict__ src,
                                                          uint32_t *__restrict__ dst,
                                                          const DevPrime *__restrict__ primes,
                                                          const MsArgs m,
                                                          const uint32_t *__restrict__ add) {
  using G = Geo<LOGN>;
  constexpr uint32_t KK = TWO ? 2 : 1;
  __shared__ double sm[G::N];
  const uint32_t tid = threadIdx.x;
  const size_t poly = blockIdx.x;
  const uint32_t *in = src + poly * KK * G::N;
  uint32_t u0[G::E], u1[G::E];
#pragma unroll
  for (int e = 0; e < G::E; ++e) {
    u0[e] = in[ridx<LOGN, true, 0>(tid, e)];
    if constexpr (TWO) u1[e] = in[G::N + ridx<LOGN, true, 0>(tid, e)];
  }
  double x[G::E];
  uint32_t y0[G::E], y1[G::E];
  const uint32_t *a = ADD && (poly & 1) ? add + (poly >> 1) * KK * G::N : nullptr;
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = (double)u0[e];
  if (ADD && a) {
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] += (double)a[ridx<LOGN, true, 0>(tid, e)];
  }
  transform<LOGN, true>(x, y0, tid, sm, primes[0]);
  if constexpr (TWO) {
    __syncthreads();  // the first transform's last LDS reads are done
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = (double)u1[e];
    if (ADD && a) {
#pragma unroll
      for (int e = 0; e < G::E; ++e) x[e] += (double)a[G::N + ridx<LOGN, true, 0>(tid, e)];
    }
    transform<LOGN, true>(x, y1, tid, sm, primes[1]);
  }
  constexpr int LAST = G::ROUNDS - 1;
  uint32_t *out = dst + poly * G::N;
#pragma unroll
  for (int e = 0; e < G::E; ++e)
    out[ridx<LOGN, true, LAST>(tid, e)] = mod_switch<TWO>(y0[e], TWO ? y1[e] : 0u, m);
}

template <bool INV, bool ADD>
hipError_t ntt_rows_dispatch(const uint32_t *src, uint32_t *dst, size_t n_rows, uint32_t K,
                             uint32_t log2n, const DevPrime *primes, const uint32_t *add,
                             hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  const dim3 grid((unsigned)n_rows);
  switch (log2n) {
    case 10: k_ntt_rows<10, INV, ADD><<<grid, Geo<10>::T, 0, s>>>(src, dst, K, primes, add); break;
    case 11: k_ntt_rows<11, INV, ADD><<<grid, Geo<11>::T, 0, s>>>(src, dst, K, primes, add); break;
    case 12: k_ntt_rows<12, INV, ADD><<<grid, Geo<12>::T, 0, s>>>(src, dst, K, primes, add); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int LOGN, bool TWO>
void intt_switch_launch(const uint32_t *src, uint32_t *dst, size_t n_polys, const DevPrime *primes,
                        const MsArgs &m, const uint32_t *add, hipStream_t s) {
  const dim3 grid((unsigned)n_polys), block(Geo<LOGN>::T);
  if (add) k_intt_switch<LOGN, TWO, true><<<grid, block, 0, s>>>(src, dst, primes, m, add);
  else k_intt_switch<LOGN, TWO, false><<<grid, block, 0, s>>>(src, dst, primes, m, nullptr);
}

template <typename T>
hipError_t lift_ntt_dispatch(const T *raw, uint32_t *out, uint32_t S, uint32_t s_valid, uint32_t C,
                             uint32_t K, uint32_t log2n, const DevPrime *primes, hipStream_t s) {
  const uint32_t rows = S * C, valid = s_valid * C;
  const dim3 grid(rows, K);
  switch (log2n) {
    case 10: k_lift_ntt<10, T><<<grid, Geo<10>::T, 0, s>>>(raw, out, rows, valid, primes); break;
    case 11: k_lift_ntt<11, T><<<grid, Geo<11>::T, 0, s>>>(raw, out, rows, valid, primes); break;
    case 12: k_lift_ntt<12, T><<<grid, Geo<12>::T, 0, s>>>(raw, out, rows, valid, primes); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ntt(uint32_t *data, size_t n_rows, uint32_t K, uint32_t log2n,
                      const DevPrime *primes, bool inverse, hipStream_t s, const uint32_t *add) {
  if (add && !inverse) return hipErrorInvalidValue;
  if (add) return ntt_rows_dispatch<true, true>(data, data, n_rows, K, log2n, primes, add, s);
  return inverse ? ntt_rows_dispatch<true, false>(data, data, n_rows, K, log2n, primes, nullptr, s)
                 : ntt_rows_dispatch<false, false>(data, data, n_rows, K, log2n, primes, nullptr, s);
}

hipError_t launch_ntt_copy(const uint32_t *src, uint32_t *dst, size_t n_rows, uint32_t K,
                           uint32_t log2n, const DevPrime *primes, hipStream_t s) {
  return ntt_rows_dispatch<false, false>(src, dst, n_rows, K, log2n, primes, nullptr, s);
}

hipError_t launch_intt_switch(const uint32_t *src, uint32_t *dst, size_t n_polys, uint32_t K,
                              const uint32_t *q, uint32_t log2n, const DevPrime *primes,
                              uint32_t bits, hipStream_t s, const uint32_t *add) {
  if (n_polys == 0) return hipSuccess;
  if (K < 1 || K > 2 || bits < 1 || bits > 32) return hipErrorInvalidValue;
  MsArgs m{};
  m.q0 = q[0];
  m.q1 = K == 2 ? q[1] : 1;
  m.Q = K == 2 ? (uint64_t)q[0] * q[1] : q[0];
  m.scale = std::ldexp(1.0, (int)bits) / (double)m.Q;
  m.q1d = (double)m.q1;
  m.inv_q1 = 1.0 / m.q1d;
  // q0^-1 mod q1 by the extended Euclidean algorithm
  int64_t r0 = m.q1, r1 = m.q0 % m.q1, t0 = 0, t1 = 1;
  while (r1 != 0) {
    const int64_t qt = r0 / r1, r2 = r0 - qt * r1, t2 = t0 - qt * t1;
    r0 = r1, r1 = r2, t0 = t1, t1 = t2;
  }
  m.c = (double)(K == 2 ? (uint32_t)((t0 % (int64_t)m.q1 + m.q1) % m.q1) : 0u);
  m.bits = bits;
  m.mask = bits == 32 ? 0xffffffffu : (1u << bits) - 1;
  const bool two = K == 2;
  switch (log2n) {
    case 10:
      if (two) intt_switch_launch<10, true>(src, dst, n_polys, primes, m, add, s);
      else intt_switch_launch<10, false>(src, dst, n_polys, primes, m, add, s);
      break;
    case 11:
      if (two) intt_switch_launch<11, true>(src, dst, n_polys, primes, m, add, s);
      else intt_switch_launch<11, false>(src, dst, n_polys, primes, m, add, s);
      break;
    case 12:
      if (two) intt_switch_launch<12, true>(src, dst, n_polys, primes, m, add, s);
      else intt_switch_launch<12, false>(src, dst, n_polys, primes, m, add, s);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lift_ntt(const uint8_t *raw, uint32_t *out, uint32_t S, uint32_t s_valid,
                           uint32_t C, uint32_t K, uint32_t log2n, const DevPrime *primes,
                           hipStream_t s) {
  return lift_ntt_dispatch<uint8_t>(raw, out, S, s_valid, C, K, log2n, primes, s);
}

hipError_t launch_lift_ntt32(const uint32_t *raw, uint32_t *out, uint32_t S, uint32_t s_valid,
                             uint32_t C, uint32_t K, uint32_t log2n, const DevPrime *primes,
                             hipStream_t s) {
  return lift_ntt_dispatch<uint32_t>(raw, out, S, s_valid, C, K, log2n, primes, s);
}

hipError_t launch_offset_ntt(const uint32_t *b, uint32_t *out, uint32_t B, uint32_t D1,
                             uint32_t Cp, uint32_t K, uint32_t log2n, const DevPrime *primes,
                             const uint32_t *delta, hipStream_t s) {
  if (B == 0) return hipSuccess;
  if (K < 1 || K > PIR_MAX_PRIMES) return hipErrorInvalidValue;
  OffsetArgs a{};
  a.D1 = D1;
  a.Cp = Cp;
  a.K = K;
  for (uint32_t k = 0; k < K; ++k) a.delta[k] = delta[k];
  const dim3 grid(B * Cp, K);
  switch (log2n) {
    case 10: k_offset_ntt<10><<<grid, Geo<10>::T, 0, s>>>(b, out, primes, a); break;
    case 11: k_offset_ntt<11><<<grid, Geo<11>::T, 0, s>>>(b, out, primes, a); break;
    case 12: k_offset_ntt<12><<<grid, Geo<12>::T, 0, s>>>(b, out, primes, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pir
