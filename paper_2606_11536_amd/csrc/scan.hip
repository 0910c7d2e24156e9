// The first-dimension scan on the int8 matrix cores (paper: Sec. 3.2 step 6;
// Sec. 4, (#RNS*N)-parallel INT32 modular GEMMs; Sec. 4.2 lazy reduction).
//
// For prime k and NTT slot t the scan is Y_t = D_t * Q_t (mod q_k), D_t the
// C x R database slice, Q_t the R x 2B query slice.  Both operands are split
// into four 7-bit limbs (x = sum_a x_a 2^(7a)); the matrix cores multiply the
// limb planes exactly:
//
//   A rows  = (database row j, limb a),  B columns = (query column, limb b),
//   acc[(j,a)][(col,b)] = sum_i d_a[j][i] * q_b[i][col]   (int32, exact).
//
// Every limb product is at most 127^2 and R <= 32768, so each sum is below
// 32768 * 16129 < 2^31 and never overflows.  The epilogue recombines
//   Y[j][col] = sum_{a,b} acc[(j,a)][(col,b)] * (2^(7(a+b)) mod q)   (mod q)
// with Shoup products, first over a inside a lane, then over b across the four
// lanes that hold b = 0..3.  Nothing is approximated: the result is the exact
// residue in [0, q).
//
// Two kernels share the database atoms:
//  * k_scan_b1 (B = 1): bandwidth-bound streaming.  v_mfma_i32_16x16x64_i8
//    with 4 database rows x 4 limbs per A operand and the two ciphertext
//    components x 4 limbs (half the B columns) per B operand.  The slot's
//    query limbs sit in LDS; database atoms stream from HBM once.
//  * k_scan_mfma (B > 1): v_mfma_i32_32x32x32_i8 over whole atoms, each wave a
//    tile of database rows x up to 64 query columns; query atoms are staged in
//    LDS per chunk of the contraction and shared by the four waves.
#include "device_util.h"
#include "pir_internal.h"

namespace pir {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr uint32_t kB1Chunk = 64;  // query ibs staged per LDS chunk (16 KiB)

struct B1Args {
  DbDesc db;
  const uint8_t *qatoms;
  uint32_t *out;
  uint32_t n_slots;   // K * N
  uint32_t jpb;       // jbs per block
  uint32_t total;     // logical blocks
};

// Reduce the lane's partial sum s over the 4 lanes b = 0..3 (lane bits 0,1).
// Input s in [0, 2q); output in [0, q).
__device__ __forceinline__ uint32_t quad_sum_mod(uint32_t s, uint32_t q) {
  s += __shfl_xor(s, 1);  // < 4q
  s += __shfl_xor(s, 2);  // < 8q
  s = csub(s, 4 * q);
  s = csub(s, 2 * q);
  return csub(s, q);
}

template <int JBW>
__global__ __launch_bounds__(256) void k_scan_b1(const B1Args a) {
  __shared__ uint4 sq[kB1Chunk * 16];
  const uint32_t L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= a.total) return;
  const DbDesc &db = a.db;
  const uint32_t slot = L % a.n_slots, jchunk = L / a.n_slots;
  const uint32_t k = slot >> db.log2n, t = slot & (db.N - 1);
  const DevPrime &P = db.primes[k];
  const uint32_t q = P.q;

  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint32_t g = lane >> 4, m = lane & 15;
  const uint32_t n_ib = db.n_ib, n_jb = db.n_jb;
  const uint32_t jb_begin = jchunk * a.jpb;
  const uint32_t jb_end = min(jb_begin + a.jpb, n_jb);
  const uint8_t *slot_atoms = db.atoms + (size_t)slot * n_jb * n_ib * kAtomBytes;
  const uint32_t lane_off = (g >> 1) * 1024 + (g & 1) * 512 + m * 16;
  const uint4 *qsrc = reinterpret_cast<const uint4 *>(a.qatoms) + (size_t)slot * n_ib * 64;

  v4i acc[JBW][2];
#pragma unroll
  for (int w = 0; w < JBW; ++w) acc[w][0] = acc[w][1] = v4i{0, 0, 0, 0};

  for (uint32_t ib0 = 0; ib0 < n_ib; ib0 += kB1Chunk) {
    const uint32_t nib = min(kB1Chunk, n_ib - ib0);  // even: R_pad is a multiple of 64
    __syncthreads();
    for (uint32_t idx = tid; idx < nib * 16; idx += 256) {
      const uint32_t ibl = idx >> 4, r = idx & 15;
      sq[idx] = qsrc[(size_t)(ib0 + ibl) * 64 + (r >> 3) * 32 + (r & 7)];
    }
    __syncthreads();
    const uint32_t nkb = nib >> 1;
#pragma unroll
    for (int w = 0; w < JBW; ++w) {
      const uint32_t jb = jb_begin + wave + 4 * w;
      if (jb >= jb_end) break;
      const uint8_t *base = slot_atoms + ((size_t)jb * n_ib + ib0) * kAtomBytes + lane_off;
#pragma unroll 4
      for (uint32_t kb = 0; kb < nkb; ++kb) {
        const v4i a0 = *reinterpret_cast<const v4i *>(base + (size_t)kb * 2048);
        const v4i a1 = *reinterpret_cast<const v4i *>(base + (size_t)kb * 2048 + 256);
        v4i bv = v4i{0, 0, 0, 0};
        if (m < 8) {
          const uint4 u = sq[(2 * kb + (g >> 1)) * 16 + (g & 1) * 8 + m];
          bv = v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
        }
        acc[w][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, bv, acc[w][0], 0, 0, 0);
        acc[w][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, bv, acc[w][1], 0, 0, 0);
      }
    }
  }

  // Epilogue.  Lane holds rows 4*(lane>>4) + r (row = 4 jl' + a, a = r) of
  // column lane & 15 (= 4 cc + b).
  const uint32_t b = lane & 3, cc = (lane >> 2) & 3, jlp = lane >> 4;
  uint32_t wv[4], wsh[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    wv[r] = P.w[r + b];
    wsh[r] = P.w_sh[r + b];
  }
  const size_t KN = (size_t)db.K * db.N;
#pragma unroll
  for (int w = 0; w < JBW; ++w) {
    const uint32_t jb = jb_begin + wave + 4 * w;
    if (jb >= jb_end) break;
#pragma unroll
    for (int jh = 0; jh < 2; ++jh) {
      uint32_t s = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) s += mul_shoup((uint32_t)acc[w][jh][r], wv[r], wsh[r], q);
      s = csub(s, 4 * q);
      s = csub(s, 2 * q);
      s = quad_sum_mod(s, q);
      const uint32_t j = jb * 8 + jh * 4 + jlp;
      if (b == 0 && cc < 2 && j < db.C) a.out[((size_t)j * 2 + cc) * KN + (size_t)k * db.N + t] = s;
    }
  }
}

// ---------------------------------------------------------------------------
constexpr uint32_t kKC = 4;   // query ibs per LDS chunk
constexpr uint32_t kCBT = 8;  // query atoms (8 columns each) per block tile

struct MfArgs {
  DbDesc db;
  const uint8_t *qatoms;
  uint32_t *out;
  uint32_t B, n_cb;
  uint32_t n_slots, n_jg, n_cbt;  // logical grid = n_cbt * n_slots * n_jg
  uint32_t total;
};

template <int JBW>
__global__ __launch_bounds__(256) void k_scan_mfma(const MfArgs a) {
  __shared__ uint4 sq[kKC * kCBT * 64];  // 32 KiB
  const uint32_t L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= a.total) return;
  const DbDesc &db = a.db;
  const uint32_t jg = L % a.n_jg;
  const uint32_t rest = L / a.n_jg;
  const uint32_t slot = rest % a.n_slots, cbt = rest / a.n_slots;
  const uint32_t k = slot >> db.log2n, t = slot & (db.N - 1);
  const DevPrime &P = db.primes[k];
  const uint32_t q = P.q;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint32_t n_ib = db.n_ib, n_jb = db.n_jb;
  const uint32_t cb0 = cbt * kCBT;
  const uint32_t ncb = min(kCBT, a.n_cb - cb0);

  uint32_t jbs[JBW];
  bool jv[JBW];
#pragma unroll
  for (int w = 0; w < JBW; ++w) {
    jbs[w] = (jg * 4 + wave) * JBW + w;
    jv[w] = jbs[w] < n_jb;
  }
  const uint8_t *slot_atoms = db.atoms + (size_t)slot * n_jb * n_ib * kAtomBytes + lane * 16;
  const uint4 *qsrc = reinterpret_cast<const uint4 *>(a.qatoms) + (size_t)slot * n_ib * a.n_cb * 64;

  v16i acc[JBW][kCBT];
#pragma unroll
  for (int w = 0; w < JBW; ++w)
#pragma unroll
    for (int c = 0; c < (int)kCBT; ++c) acc[w][c] = v16i{};

  for (uint32_t ib0 = 0; ib0 < n_ib; ib0 += kKC) {
    const uint32_t nib = min(kKC, n_ib - ib0);
    __syncthreads();
    for (uint32_t idx = tid; idx < kKC * kCBT * 64; idx += 256) {
      const uint32_t kk = idx / (kCBT * 64), c = (idx / 64) % kCBT, l = idx & 63;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (kk < nib && c < ncb) v = qsrc[((size_t)(ib0 + kk) * a.n_cb + cb0 + c) * 64 + l];
      sq[idx] = v;
    }
    __syncthreads();
    for (uint32_t kk = 0; kk < nib; ++kk) {
      v4i av[JBW];
#pragma unroll
      for (int w = 0; w < JBW; ++w) {
        av[w] = v4i{0, 0, 0, 0};
        if (jv[w])
          av[w] = *reinterpret_cast<const v4i *>(slot_atoms +
                                                 ((size_t)jbs[w] * n_ib + ib0 + kk) * kAtomBytes);
      }
#pragma unroll
      for (int c = 0; c < (int)kCBT; ++c) {
        if ((uint32_t)c >= ncb) break;
        const uint4 u = sq[(kk * kCBT + c) * 64 + lane];
        const v4i bv = v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
#pragma unroll
        for (int w = 0; w < JBW; ++w)
          acc[w][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av[w], bv, acc[w][c], 0, 0, 0);
      }
    }
  }

  // Epilogue.  32x32 result: lane holds column lane & 31 (= 4 cc + b) and, in
  // register r, row 8*(r>>2) + 4*(lane>>5) + (r&3)  (row = 4 jl + a).
  const uint32_t b = lane & 3, cc = (lane >> 2) & 7, hi = lane >> 5;
  uint32_t wv[4], wsh[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    wv[r] = P.w[r + b];
    wsh[r] = P.w_sh[r + b];
  }
  const size_t KN = (size_t)db.K * db.N;
  const uint32_t ncol = 2 * a.B;
#pragma unroll
  for (int w = 0; w < JBW; ++w) {
    if (!jv[w]) continue;
#pragma unroll
    for (int c = 0; c < (int)kCBT; ++c) {
      if ((uint32_t)c >= ncb) break;
      const uint32_t col = (cb0 + c) * 8 + cc;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        uint32_t s = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          s += mul_shoup((uint32_t)acc[w][c][4 * qq + r], wv[r], wsh[r], q);
        s = csub(s, 4 * q);
        s = csub(s, 2 * q);
        s = quad_sum_mod(s, q);
        const uint32_t j = jbs[w] * 8 + 2 * qq + hi;
        if (b == 0 && j < db.C && col < ncol)
          a.out[(((size_t)(col >> 1) * db.C + j) * 2 + (col & 1)) * KN + (size_t)k * db.N + t] = s;
      }
    }
  }
}

inline uint32_t round8(uint32_t x) { return (x + 7) / 8 * 8; }

}  // namespace

hipError_t launch_scan(const ScanJob &job, int num_cus, hipStream_t s) {
  (void)num_cus;
  const DbDesc &db = job.db;
  const uint32_t n_slots = db.K * db.N;
  if (job.B == 1) {
    constexpr int JBW = 8;
    B1Args a;
    a.db = db;
    a.qatoms = job.qatoms;
    a.out = job.out;
    a.n_slots = n_slots;
    a.jpb = 4 * JBW;
    const uint32_t n_jchunks = (db.n_jb + a.jpb - 1) / a.jpb;
    a.total = n_slots * n_jchunks;
    k_scan_b1<JBW><<<round8(a.total), 256, 0, s>>>(a);
    return hipGetLastError();
  }
  constexpr int JBW = 1;
  MfArgs a;
  a.db = db;
  a.qatoms = job.qatoms;
  a.out = job.out;
  a.B = job.B;
  a.n_cb = (2 * job.B + kCB - 1) / kCB;
  a.n_slots = n_slots;
  a.n_jg = (db.n_jb + 4 * JBW - 1) / (4 * JBW);
  a.n_cbt = (a.n_cb + kCBT - 1) / kCBT;
  a.total = a.n_cbt * n_slots * a.n_jg;
  k_scan_mfma<JBW><<<round8(a.total), 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace pir
