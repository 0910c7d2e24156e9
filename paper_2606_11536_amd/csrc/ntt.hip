// Negacyclic NTT / INTT over Z_q[X]/(X^N + 1), q < 2^28, N in {1024, 2048, 4096}
// (paper: Sec. 2.3; single-kernel transform of Sec. 4.3).
//
// One 256-thread workgroup transforms one residue row of N values.  Each
// thread keeps E = N/256 values in registers and performs log2(E) radix-2
// stages on them before the block exchanges values through LDS; the
// log2(N) stages therefore take ceil(log2 N / log2 E) register rounds.
//
// Forward: Cooley-Tukey stages with half-sizes N/2, N/4, ..., 1; the stage
// with half-size h uses twiddle psi^brv(N/(2h) + x/(2h)) for the pair
// (x, x + h).  Natural-order input, output slot t = a(psi^(2 brv(t) + 1)).
// Inverse: Gentleman-Sande stages with half-sizes 1, 2, ..., N/2 and the
// inverse twiddles, then the factor N^-1.
//
// Arithmetic: Shoup multiplication by precomputed twiddle quotients; forward
// values stay lazily in [0, 4q) and inverse values in [0, 2q) (both < 2^30),
// reduced to [0, q) once at the end.
#include "device_util.h"
#include "pir_internal.h"

namespace pir {
namespace {

constexpr int kThreads = 256;

template <int LOGN>
struct Geo {
  static constexpr int N = 1 << LOGN;
  static constexpr int LE = LOGN - 8;  // log2 of values per thread
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

// Index of register e in round r for thread tid.
template <int LOGN, bool INV, int R>
__device__ __forceinline__ uint32_t ridx(uint32_t tid, int e) {
  using G = Geo<LOGN>;
  constexpr int S = G::s(R, INV);
  constexpr int LL = G::logL(R, INV);
  const uint32_t g = (uint32_t)e >> S;
  const uint32_t ep = (uint32_t)e & ((1u << S) - 1);
  const uint32_t gid = tid + g * kThreads;
  const uint32_t x0 = ((gid >> LL) << (LL + S)) + (gid & ((1u << LL) - 1));
  return x0 + (ep << LL);
}

template <int LOGN, bool INV, int R>
__device__ __forceinline__ void round_compute(uint32_t (&x)[Geo<LOGN>::E], uint32_t tid,
                                              const uint32_t *__restrict__ tw,
                                              const uint32_t *__restrict__ twsh, uint32_t q) {
  using G = Geo<LOGN>;
  constexpr int S = G::s(R, INV);
  constexpr int LL = G::logL(R, INV);
  const uint32_t q2 = 2 * q;
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
      const uint32_t w = tw[ti], wsh = twsh[ti];
      const uint32_t X = x[e], Y = x[f];
      if (!INV) {
        const uint32_t Xr = csub(X, q2);
        const uint32_t T = mul_shoup(Y, w, wsh, q);
        x[e] = Xr + T;
        x[f] = Xr - T + q2;
      } else {
        x[e] = csub(X + Y, q2);
        x[f] = mul_shoup(X - Y + q2, w, wsh, q);
      }
    }
  }
}

template <int LOGN, bool INV, int R>
__device__ __forceinline__ void rounds_from(uint32_t (&x)[Geo<LOGN>::E], uint32_t tid,
                                            uint32_t *sm, const uint32_t *tw,
                                            const uint32_t *twsh, uint32_t q) {
  using G = Geo<LOGN>;
  round_compute<LOGN, INV, R>(x, tid, tw, twsh, q);
  if constexpr (R + 1 < G::ROUNDS) {
    if (R > 0) __syncthreads();  // the previous round's reads are done
#pragma unroll
    for (int e = 0; e < G::E; ++e) sm[ridx<LOGN, INV, R>(tid, e)] = x[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = sm[ridx<LOGN, INV, R + 1>(tid, e)];
    rounds_from<LOGN, INV, R + 1>(x, tid, sm, tw, twsh, q);
  }
}

// Transform the values in x (loaded with round-0 indexing); on return x holds
// canonical residues in [0, q) laid out with last-round indexing.
template <int LOGN, bool INV>
__device__ __forceinline__ void transform(uint32_t (&x)[Geo<LOGN>::E], uint32_t tid,
                                          uint32_t *sm, const DevPrime &P) {
  constexpr int N = Geo<LOGN>::N;
  const uint32_t q = P.q;
  const uint32_t *tw = P.tw + (INV ? 2 * N : 0);
  const uint32_t *twsh = P.tw + (INV ? 3 * N : N);
  rounds_from<LOGN, INV, 0>(x, tid, sm, tw, twsh, q);
#pragma unroll
  for (int e = 0; e < Geo<LOGN>::E; ++e) {
    uint32_t v = x[e];
    if (!INV) {
      v = csub(v, 2 * q);
      v = csub(v, q);
    } else {
      v = csub(mul_shoup(v, P.ninv, P.ninv_sh, q), q);
    }
    x[e] = v;
  }
}

template <int LOGN, bool INV>
__global__ __launch_bounds__(kThreads) void k_ntt_rows(const uint32_t *__restrict__ src,
                                                       uint32_t *__restrict__ dst, uint32_t K,
                                                       const DevPrime *__restrict__ primes) {
  using G = Geo<LOGN>;
  __shared__ uint32_t sm[G::N];
  const uint32_t tid = threadIdx.x;
  const size_t row = blockIdx.x;
  const DevPrime &P = primes[row % K];
  const uint32_t *in = src + row * G::N;
  uint32_t *out = dst + row * G::N;
  uint32_t x[G::E];
#pragma unroll
  for (int e = 0; e < G::E; ++e) x[e] = in[ridx<LOGN, INV, 0>(tid, e)];
  transform<LOGN, INV>(x, tid, sm, P);
  constexpr int LAST = G::ROUNDS - 1;
#pragma unroll
  for (int e = 0; e < G::E; ++e) out[ridx<LOGN, INV, LAST>(tid, e)] = x[e];
}

// raw: [rows][N] uint8 (rows = S*C of the slab); out: [K][rows][N].
template <int LOGN>
__global__ __launch_bounds__(kThreads) void k_lift_ntt(const uint8_t *__restrict__ raw,
                                                       uint32_t *__restrict__ out, uint32_t rows,
                                                       uint32_t valid_rows,
                                                       const DevPrime *__restrict__ primes) {
  using G = Geo<LOGN>;
  __shared__ uint32_t sm[G::N];
  const uint32_t tid = threadIdx.x;
  const uint32_t row = blockIdx.x;
  const uint32_t k = blockIdx.y;
  const DevPrime &P = primes[k];
  uint32_t x[G::E];
  if (row < valid_rows) {
    const uint8_t *in = raw + (size_t)row * G::N;
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = in[ridx<LOGN, false, 0>(tid, e)];
  } else {
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = 0;
  }
  transform<LOGN, false>(x, tid, sm, P);
  uint32_t *o = out + ((size_t)k * rows + row) * G::N;
  constexpr int LAST = G::ROUNDS - 1;
#pragma unroll
  for (int e = 0; e < G::E; ++e) o[ridx<LOGN, false, LAST>(tid, e)] = x[e];
}

template <bool INV>
hipError_t ntt_rows_dispatch(const uint32_t *src, uint32_t *dst, size_t n_rows, uint32_t K,
                             uint32_t log2n, const DevPrime *primes, hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  const dim3 grid((unsigned)n_rows), block(kThreads);
  switch (log2n) {
    case 10: k_ntt_rows<10, INV><<<grid, block, 0, s>>>(src, dst, K, primes); break;
    case 11: k_ntt_rows<11, INV><<<grid, block, 0, s>>>(src, dst, K, primes); break;
    case 12: k_ntt_rows<12, INV><<<grid, block, 0, s>>>(src, dst, K, primes); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ntt(uint32_t *data, size_t n_rows, uint32_t K, uint32_t log2n,
                      const DevPrime *primes, bool inverse, hipStream_t s) {
  return inverse ? ntt_rows_dispatch<true>(data, data, n_rows, K, log2n, primes, s)
                 : ntt_rows_dispatch<false>(data, data, n_rows, K, log2n, primes, s);
}

hipError_t launch_ntt_copy(const uint32_t *src, uint32_t *dst, size_t n_rows, uint32_t K,
                           uint32_t log2n, const DevPrime *primes, hipStream_t s) {
  return ntt_rows_dispatch<false>(src, dst, n_rows, K, log2n, primes, s);
}

hipError_t launch_lift_ntt(const uint8_t *raw, uint32_t *out, uint32_t S, uint32_t s_valid,
                           uint32_t C, uint32_t K, uint32_t log2n, const DevPrime *primes,
                           hipStream_t s) {
  const uint32_t rows = S * C, valid = s_valid * C;
  const dim3 grid(rows, K), block(kThreads);
  switch (log2n) {
    case 10: k_lift_ntt<10><<<grid, block, 0, s>>>(raw, out, rows, valid, primes); break;
    case 11: k_lift_ntt<11><<<grid, block, 0, s>>>(raw, out, rows, valid, primes); break;
    case 12: k_lift_ntt<12><<<grid, block, 0, s>>>(raw, out, rows, valid, primes); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pir
