// Scalar-HE database GEMM mod 2^32 (paper: Sec. 4.1, INT8-INT32 GEMM on the
// matrix engines; Sec. 2, the SimplePIR online step):
//
//   out[b][r] = sum_c DB[r][c] * Q[b][c]   (mod 2^32),
//
// DB an int8 D1 x D0 matrix, Q a batch of B uint32 query vectors.
//
// Each query word is split into four balanced signed digits,
//   q = d0 + 2^8 d1 + 2^16 d2 + 2^24 d3 (mod 2^32), d_k in [-128, 127]
// (d0 is the low byte read as a signed byte; the rest of q minus d0 is
// divided by 2^8 and split the same way), so that every digit is an int8
// operand of v_mfma_i32_32x32x32_i8.  Products are at most 2^14 in magnitude,
// so sums over D0 < 2^17 terms stay below 2^31: every int32 accumulator is
// exact.  The epilogue shifts digit k's sum by 8k bits and adds the four
// mod 2^32.
//
// Layouts (1 KiB atoms, lane l = 32 g + x owns bytes [16 l, 16 l + 16)):
//  * database atom (rb, kb): DB[32 rb + x][32 kb + 16 g + e], e < 16; atom
//    order [rb][kb] with kb padded to a multiple of 8 and rows past D1,
//    columns past D0 zero;
//  * query atom (kb, cb): digit (x & 3) of Q[8 cb + (x >> 2)][32 kb + 16 g + e];
//    atom order [kb][cb] with cb padded to a multiple of 4, zero past B.
// As in the scan, lane l feeds the same 16 contraction indices to the A and
// B operands.  The 32 x 32 result holds column lane & 31 (= 4 b' + k) and,
// in register r, row 8 (r >> 2) + 4 (lane >> 5) + (r & 3): the four digits
// of one output lie in one quad of lanes.
#include <hip/hip_ext.h>

#include "device_util.h"
#include "pir_internal.h"

namespace pir {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// One atom per 64 threads: lane l gathers its 16 database bytes.
__global__ __launch_bounds__(256) void k_sdb_pack(const int8_t *__restrict__ db,
                                                  uint8_t *__restrict__ atoms, uint32_t D1,
                                                  uint32_t D0, uint32_t n_kb, uint32_t n_atoms) {
  const uint32_t atom = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (atom >= n_atoms) return;
  const uint32_t rb = atom / n_kb, kb = atom % n_kb;
  const uint32_t r = rb * 32 + (l & 31), c0 = kb * 32 + (l >> 5) * 16;
  uint32_t w[4] = {0, 0, 0, 0};
  if (r < D1) {
    const int8_t *row = db + (size_t)r * D0;
#pragma unroll
    for (int e = 0; e < 16; ++e)
      if (c0 + e < D0) w[e >> 2] |= (uint32_t)(uint8_t)row[c0 + e] << (8 * (e & 3));
  }
  reinterpret_cast<uint4 *>(atoms)[(size_t)atom * 64 + l] = make_uint4(w[0], w[1], w[2], w[3]);
}

// Digit k (0..3) of the balanced signed split of q, as a byte.
__device__ __forceinline__ uint32_t digit(uint32_t q, uint32_t k) {
  uint32_t d = 0;
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) {
    const int32_t s = (int32_t)(int8_t)(uint8_t)(q & 255u);  // low byte, signed
    if (i == k) d = (uint32_t)(uint8_t)s;
    q = (q - (uint32_t)s) >> 8;                                // exact: q - s = 0 mod 2^8
  }
  return d;
}

// One query atom per 64 threads.
__global__ __launch_bounds__(256) void k_sq_pack(const uint32_t *__restrict__ q,
                                                 uint8_t *__restrict__ atoms, uint32_t B,
                                                 uint32_t D0, uint32_t n_cb, uint32_t n_atoms) {
  const uint32_t atom = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (atom >= n_atoms) return;
  const uint32_t kb = atom / n_cb, cb = atom % n_cb;
  const uint32_t x = l & 31, b = cb * 8 + (x >> 2), k = x & 3, c0 = kb * 32 + (l >> 5) * 16;
  uint32_t w[4] = {0, 0, 0, 0};
  if (b < B) {
    const uint32_t *row = q + (size_t)b * D0;
#pragma unroll
    for (int e = 0; e < 16; ++e)
      if (c0 + e < D0) w[e >> 2] |= digit(row[c0 + e], k) << (8 * (e & 3));
  }
  reinterpret_cast<uint4 *>(atoms)[(size_t)atom * 64 + l] = make_uint4(w[0], w[1], w[2], w[3]);
}

struct SgArgs {
  const uint8_t *db;     // database atoms [n_rb][n_kb]
  const uint8_t *q;      // query atoms [n_kb][n_cb]
  uint32_t *out;         // [B][D1]
  uint32_t D1, B, n_rb, n_kb, n_cb, n_ct, n_rg, total;
};

// Block = NW waves (four: one per SIMD; eight: two per SIMD); wave w of row
// group rg owns row blocks (NW rg + w) JBW .. + JBW - 1 and the CBW column
// blocks of column tile ct.  The column tiles of
// one row group are adjacent logical blocks, so they run together and read
// the group's database atoms from HBM once.  Database atoms come through a
// register ring D k-blocks deep (the loads of the last D steps are clamped to
// the last k-block: valid memory, never used).  Query atoms are shared
// through LDS: per chunk of KC k-blocks the NW waves load the chunk's
// KC x CBW query atoms once (a share each, into registers), write them to
// one of two LDS buffers and meet at a barrier; every wave then reads its B
// operands from LDS.  The loads of chunk n + 1 go out at the start of chunk n
// and are written at its end, into the buffer last read in chunk n - 1.
template <int JBW, int CBW, int D, int KC, int NW>
__global__ __launch_bounds__(64 * NW) void k_sgemm(const SgArgs a) {
  static_assert(KC % D == 0 && (KC * CBW) % NW == 0, "chunk shape");
  constexpr int kPer = KC * CBW / NW;  // staged atoms per wave per chunk
  __shared__ uint4 sq[2][KC * CBW * 64];
  const uint32_t L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= a.total) return;
  const uint32_t ct = L % a.n_ct, rg = L / a.n_ct;
  const uint32_t lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t rb0 = (rg * NW + wave) * JBW, cb0 = ct * CBW, nkb = a.n_kb;
  const v4i *pa[JBW];
#pragma unroll
  for (int w = 0; w < JBW; ++w) {
    const uint32_t rb = rb0 + w < a.n_rb ? rb0 + w : a.n_rb - 1;  // past the end: discarded
    pa[w] = reinterpret_cast<const v4i *>(a.db + (size_t)rb * nkb * kAtomBytes) + lane;
  }
  const uint4 *qa = reinterpret_cast<const uint4 *>(a.q) + lane;
  // staged atom i = wave + NW r of a chunk is (kk, c) = (i / CBW, i % CBW)
  auto stage_load = [&](uint32_t chunk, uint4 (&st)[kPer]) {
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const uint32_t i = wave + NW * r, kb = chunk * KC + i / CBW;
      const uint32_t kbc = kb < nkb ? kb : nkb - 1;  // past the end: never read
      st[r] = qa[((size_t)kbc * a.n_cb + cb0 + i % CBW) * 64];
    }
  };
  auto stage_store = [&](uint32_t buf, const uint4 (&st)[kPer]) {
#pragma unroll
    for (int r = 0; r < kPer; ++r) sq[buf][(wave + NW * r) * 64 + lane] = st[r];
  };

  v16i acc[JBW][CBW];
#pragma unroll
  for (int w = 0; w < JBW; ++w)
#pragma unroll
    for (int c = 0; c < CBW; ++c) acc[w][c] = v16i{};
  v4i ra[D][JBW];
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int w = 0; w < JBW; ++w) ra[d][w] = __builtin_nontemporal_load(pa[w] + (size_t)d * 64);
  uint4 st[kPer];
  stage_load(0, st);
  stage_store(0, st);
  __syncthreads();
  const uint32_t nch = nkb / KC;
  for (uint32_t ch = 0; ch < nch; ++ch) {
    const uint32_t buf = ch & 1;
    stage_load(ch + 1, st);
    for (uint32_t kk0 = 0; kk0 < (uint32_t)KC; kk0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const uint32_t kb = ch * KC + kk0 + d;
        v4i bq[CBW];
#pragma unroll
        for (int c = 0; c < CBW; ++c) {
          const uint4 u = sq[buf][((kk0 + d) * CBW + c) * 64 + lane];
          bq[c] = v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
        }
#pragma unroll
        for (int w = 0; w < JBW; ++w)
#pragma unroll
          for (int c = 0; c < CBW; ++c)
            acc[w][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ra[d][w], bq[c], acc[w][c], 0, 0, 0);
        const uint32_t nk = kb + D < nkb ? kb + D : nkb - 1;
#pragma unroll
        for (int w = 0; w < JBW; ++w) ra[d][w] = __builtin_nontemporal_load(pa[w] + (size_t)nk * 64);
      }
    }
    stage_store(buf ^ 1, st);
    __syncthreads();
  }

  const uint32_t k = lane & 3, bq8 = (lane >> 2) & 7, hi = lane >> 5;
#pragma unroll
  for (int w = 0; w < JBW; ++w) {
    const uint32_t rb = rb0 + w;
#pragma unroll
    for (int c = 0; c < CBW; ++c) {
      const uint32_t b = (cb0 + c) * 8 + bq8;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint32_t v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          uint32_t s = (uint32_t)acc[w][c][4 * j + i] << (8 * k);
          s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0xB1, 0xF, 0xF, false);
          s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x4E, 0xF, 0xF, false);
          v[i] = s;
        }
        const uint32_t mine = k == 0 ? v[0] : k == 1 ? v[1] : k == 2 ? v[2] : v[3];
        const uint32_t row = rb * 32 + 8 * j + 4 * hi + k;
        if (rb < a.n_rb && b < a.B && row < a.D1) a.out[(size_t)b * a.D1 + row] = mine;
      }
    }
  }
}

template <int JBW, int CBW, int D, int KC, int NW>
hipError_t run_sgemm(const uint8_t *db, const uint8_t *q, uint32_t *out, uint32_t D1,
                         uint32_t B, uint32_t n_rb, uint32_t n_kb, uint32_t n_cb, hipStream_t s,
                         hipEvent_t e0, hipEvent_t e1) {
  SgArgs a{};
  a.db = db;
  a.q = q;
  a.out = out;
  a.D1 = D1;
  a.B = B;
  a.n_rb = n_rb;
  a.n_kb = n_kb;
  a.n_cb = n_cb;
  a.n_ct = ((B + 7) / 8 + CBW - 1) / CBW;
  a.n_rg = (n_rb + NW * JBW - 1) / (NW * JBW);
  a.total = a.n_rg * a.n_ct;
  const uint32_t grid = (a.total + 7) / 8 * 8;
  hipExtLaunchKernelGGL(k_sgemm<JBW, CBW, D, KC, NW>, dim3(grid), dim3(64 * NW), 0, s, e0, e1, 0,
                        a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sdb_pack(const int8_t *db, uint8_t *atoms, uint32_t D1, uint32_t D0,
                           uint32_t n_rb, uint32_t n_kb, hipStream_t s) {
  const uint32_t n_atoms = n_rb * n_kb;
  if (n_atoms == 0) return hipSuccess;
  k_sdb_pack<<<(n_atoms + 3) / 4, 256, 0, s>>>(db, atoms, D1, D0, n_kb, n_atoms);
  return hipGetLastError();
}

hipError_t launch_sq_pack(const uint32_t *q, uint8_t *atoms, uint32_t B, uint32_t D0,
                          uint32_t n_kb, uint32_t n_cb, hipStream_t s) {
  const uint32_t n_atoms = n_kb * n_cb;
  if (n_atoms == 0) return hipSuccess;
  k_sq_pack<<<(n_atoms + 3) / 4, 256, 0, s>>>(q, atoms, B, D0, n_cb, n_atoms);
  return hipGetLastError();
}

hipError_t launch_sgemm(const uint8_t *db, const uint8_t *q, uint32_t *out, uint32_t D1,
                        uint32_t B, uint32_t n_rb, uint32_t n_kb, uint32_t n_cb, hipStream_t s,
                        hipEvent_t e0, hipEvent_t e1) {
  const uint32_t used = (B + 7) / 8;  // column blocks that hold queries
  if (n_kb % 8 != 0 || n_cb % 4 != 0 || n_rb == 0 || used == 0 || used > n_cb)
    return hipErrorInvalidValue;
  if (used <= 1) return run_sgemm<2, 1, 8, 8, 4>(db, q, out, D1, B, n_rb, n_kb, n_cb, s, e0, e1);
  if (used <= 2) return run_sgemm<2, 2, 8, 8, 4>(db, q, out, D1, B, n_rb, n_kb, n_cb, s, e0, e1);
  // from three column blocks up, eight waves (two per SIMD) share each query
  // chunk: 16 GiB database, B = 32: 3.04 -> 2.91 ms (B = 1 and 16 are 1 %
  // faster with four)
  return run_sgemm<2, 4, 8, 8, 8>(db, q, out, D1, B, n_rb, n_kb, n_cb, s, e0, e1);
}

}  // namespace pir
