// Layout transposition between polynomial-major NTT form and the slot-major,
// limb-planar atoms the scan consumes (paper: Sec. 4.2, layout
// transposition between NTT-friendly and GEMM-friendly layouts).
//
// Each packing workgroup stages a 32 (i) x 8 (j or column) x 32 (t) tile of
// residues in LDS -- read as 128-byte runs along t -- and writes 32 whole
// 1 KiB atoms, one per slot t, so both sides of the transposition move full
// contiguous lines.
#include <algorithm>

#include "device_util.h"
#include "pir_internal.h"

namespace pir {
namespace {

constexpr int kPad = 33;  // LDS row pitch (words) of the t dimension

// slab: [K][S][C][N] NTT-form residues of rows i0 .. i0 + S - 1.
__global__ __launch_bounds__(256) void k_pack_db(const uint32_t *__restrict__ slab,
                                                 uint8_t *__restrict__ atoms, uint32_t ib_first,
                                                 uint32_t S, uint32_t C, uint32_t N,
                                                 uint32_t n_jb, uint32_t n_ib) {
  __shared__ uint32_t lds[32 * 8 * kPad];
  const uint32_t tid = threadIdx.x;
  const uint32_t t0 = blockIdx.x * 32;
  const uint32_t jb = blockIdx.y;
  const uint32_t ib_per_slab = S / 32;
  const uint32_t k = blockIdx.z / ib_per_slab;
  const uint32_t ibl = blockIdx.z % ib_per_slab;
  const uint32_t ib = ib_first + ibl;
  if (ib >= n_ib) return;  // slab rows past R_pad: nothing to write

  const uint32_t tt = tid & 31, p = tid >> 5;
#pragma unroll 4
  for (uint32_t r = 0; r < 32; ++r) {
    const uint32_t pi = p + 8 * r;
    const uint32_t il = pi >> 3, jl = pi & 7;
    const uint32_t j = jb * 8 + jl;
    uint32_t v = 0;
    if (j < C) v = slab[(((size_t)k * S + ibl * 32 + il) * C + j) * N + t0 + tt];
    lds[(il * 8 + jl) * kPad + tt] = v;
  }
  __syncthreads();
  uint4 *out = reinterpret_cast<uint4 *>(atoms);
#pragma unroll 2
  for (uint32_t r = 0; r < 8; ++r) {
    const uint32_t w = tid + 256 * r;
    const uint32_t tl = w >> 6, lane = w & 63;
    const uint32_t g = lane >> 5, m = lane & 31, jl = m >> 2, a = m & 3;
    uint32_t word[4];
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) {
      uint32_t acc = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t v = lds[((16 * g + 4 * q4 + e) * 8 + jl) * kPad + tl];
        acc |= ((v >> (7 * a)) & 127u) << (8 * e);
      }
      word[q4] = acc;
    }
    const size_t atom = (((size_t)k * N + t0 + tl) * n_jb + jb) * n_ib + ib;
    out[atom * 64 + lane] = make_uint4(word[0], word[1], word[2], word[3]);
  }
}

// Canonical read-back: out[ii][jj][k][t] for rows i0 + ii, columns j0 + jj.
__global__ void k_read_db(DbDesc db, uint32_t i0, uint32_t ni, uint32_t j0, uint32_t nj,
                          uint32_t *__restrict__ out) {
  const size_t total = (size_t)ni * nj * db.K * db.N;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const uint32_t t = idx % db.N;
    size_t rest = idx / db.N;
    const uint32_t k = rest % db.K;
    rest /= db.K;
    const uint32_t jj = rest % nj;
    const uint32_t ii = rest / nj;
    const uint32_t i = i0 + ii, j = j0 + jj;
    const size_t atom = (((size_t)k * db.N + t) * db.n_jb + j / 8) * db.n_ib + i / 32;
    const uint32_t lane0 = ((i % 32) >> 4) * 32 + (j % 8) * 4;
    const uint8_t *p = db.atoms + atom * kAtomBytes + (i % 16);
    uint32_t v = 0;
#pragma unroll
    for (uint32_t a = 0; a < 4; ++a) v |= (uint32_t)p[(lane0 + a) * 16] << (7 * a);
    out[idx] = v;
  }
}

// q: [B][R][2][K][N] NTT form -> query atoms [K][N][n_ib][n_cb].
__global__ __launch_bounds__(256) void k_pack_query(const uint32_t *__restrict__ q,
                                                    uint8_t *__restrict__ qatoms, uint32_t B,
                                                    uint32_t R, uint32_t N, uint32_t K,
                                                    uint32_t n_ib, uint32_t n_cb) {
  __shared__ uint32_t lds[32 * 8 * kPad];
  const uint32_t tid = threadIdx.x;
  const uint32_t t0 = blockIdx.x * 32;
  const uint32_t ib = blockIdx.y;
  const uint32_t k = blockIdx.z / n_cb, cb = blockIdx.z % n_cb;
  const uint32_t tt = tid & 31, p = tid >> 5;
  const uint32_t ncol = 2 * B;
  // All 32 loads of a thread are issued before the first is used (the tile's
  // 32 KiB in flight at once); rows past R and columns past 2B read element 0
  // and are masked to zero, so no load sits under a branch.
  uint32_t v[32];
#pragma unroll
  for (uint32_t r = 0; r < 32; ++r) {
    const uint32_t pi = p + 8 * r;
    const uint32_t il = pi >> 3, cc = pi & 7;
    const uint32_t i = ib * 32 + il, col = cb * 8 + cc;
    const bool ok = i < R && col < ncol;
    const size_t at = ((((size_t)(col >> 1) * R + i) * 2 + (col & 1)) * K + k) * N + t0 + tt;
    v[r] = q[ok ? at : 0] & (ok ? ~0u : 0u);
  }
#pragma unroll
  for (uint32_t r = 0; r < 32; ++r) {
    const uint32_t pi = p + 8 * r;
    lds[((pi >> 3) * 8 + (pi & 7)) * kPad + tt] = v[r];
  }
  __syncthreads();
  uint4 *out = reinterpret_cast<uint4 *>(qatoms);
#pragma unroll
  for (uint32_t r = 0; r < 8; ++r) {
    const uint32_t w = tid + 256 * r;
    const uint32_t tl = w >> 6, lane = w & 63;
    const uint32_t g = lane >> 5, n = lane & 31, cc = n >> 2, b = n & 3;
    uint32_t word[4];
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) {
      uint32_t acc = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t v = lds[((16 * g + 4 * q4 + e) * 8 + cc) * kPad + tl];
        acc |= ((v >> (7 * b)) & 127u) << (8 * e);
      }
      word[q4] = acc;
    }
    const size_t atom = (((size_t)k * N + t0 + tl) * n_ib + ib) * n_cb + cb;
    out[atom * 64 + lane] = make_uint4(word[0], word[1], word[2], word[3]);
  }
}

// One query [R][2][K][N] into its columns 2 col_slot + comp of column-block-
// major query atoms [K][N][n_cb][n_ib] (the server's layout).  In an atom the
// query owns lanes 32 half + 4 cc + b for cc = cc0, cc0 + 1 and limbs b < 4:
// two 128-byte lines, one per half.  Column-block-major order puts a slot's
// n_ib atoms of one column block next to each other, so the lines a block
// writes for one slot lie within a few KiB.
// Block = (32 slots, kPqIB row blocks, prime k): rows i of both components are
// staged in LDS as 128-byte runs along t, then every line is written by 8
// lanes, 16 bytes each.
constexpr uint32_t kPqIB = 4;  // row blocks per workgroup

__global__ __launch_bounds__(256) void k_pack_query_slot(const uint32_t *__restrict__ q,
                                                         uint8_t *__restrict__ qatoms,
                                                         uint32_t col_slot, uint32_t n_cb,
                                                         uint32_t R, uint32_t N, uint32_t K,
                                                         uint32_t n_ib) {
  // row r = (ibl 32 + il) 2 + comp, t along the pitch
  __shared__ uint32_t lds[kPqIB * 32 * 2 * kPad];
  const uint32_t tid = threadIdx.x;
  const uint32_t t0 = blockIdx.x * 32, ib0 = blockIdx.y * kPqIB, k = blockIdx.z;
  const uint32_t tt = tid & 31, p = tid >> 5;
  uint32_t v[32];
#pragma unroll
  for (uint32_t r = 0; r < 32; ++r) {
    const uint32_t row = p + 8 * r;
    const uint32_t comp = row & 1, il = (row >> 1) & 31, ibl = row >> 6;
    const uint32_t i = (ib0 + ibl) * 32 + il;
    const bool ok = i < R;
    const size_t at = (((size_t)i * 2 + comp) * K + k) * N + t0 + tt;
    v[r] = q[ok ? at : 0] & (ok ? ~0u : 0u);
  }
#pragma unroll
  for (uint32_t r = 0; r < 32; ++r) lds[(p + 8 * r) * kPad + tt] = v[r];
  __syncthreads();
  const uint32_t cb = (2 * col_slot) / kCB, cc0 = (2 * col_slot) % kCB;
  uint4 *out = reinterpret_cast<uint4 *>(qatoms);
  // line = (tl, ibl, half), half fastest: a wave's 8 lines are one slot's
  // 4 consecutive atoms, both halves
#pragma unroll
  for (uint32_t rr = 0; rr < 8; ++rr) {
    const uint32_t w = tid + 256 * rr;
    const uint32_t part = w & 7, line = w >> 3;
    const uint32_t half = line & 1, ibl = (line >> 1) & (kPqIB - 1), tl = line >> 3;
    const uint32_t comp = part >> 2, b = part & 3;
    uint32_t word[4];
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) {
      uint32_t acc = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t row = (ibl * 32 + half * 16 + 4 * q4 + e) * 2 + comp;
        acc |= ((lds[row * kPad + tl] >> (7 * b)) & 127u) << (8 * e);
      }
      word[q4] = acc;
    }
    if (ib0 + ibl < n_ib) {
      const size_t atom = (((size_t)k * N + t0 + tl) * n_cb + cb) * n_ib + ib0 + ibl;
      out[atom * 64 + half * 32 + cc0 * 4 + part] = make_uint4(word[0], word[1], word[2], word[3]);
    }
  }
}

// Slot-major answers -> polynomial-major: out[p][s] = sm[s * p_stride + p0 + p].
// A block moves a 64 (slots) x 64 (polynomials) tile through LDS, reading and
// writing 256-byte rows.
__global__ __launch_bounds__(256) void k_unpack_answers(const uint32_t *__restrict__ sm,
                                                        uint32_t p_stride, uint32_t p0, uint32_t P,
                                                        uint32_t KN, uint32_t *__restrict__ out) {
  __shared__ uint32_t tile[64][65];
  const uint32_t pb = blockIdx.x * 64, s0 = blockIdx.y * 64;
  const uint32_t tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  // all 16 loads in flight before the first LDS store; polynomials past P
  // read a valid word and are masked
  const uint32_t p = pb + tx;
  const bool ok = p < P;
  uint32_t v[16];
#pragma unroll
  for (uint32_t r = 0; r < 16; ++r)
    v[r] = sm[(size_t)(s0 + ty + 4 * r) * p_stride + p0 + (ok ? p : 0)] & (ok ? ~0u : 0u);
#pragma unroll
  for (uint32_t r = 0; r < 16; ++r) tile[ty + 4 * r][tx] = v[r];
  __syncthreads();
#pragma unroll
  for (uint32_t r = 0; r < 16; ++r) {
    const uint32_t pr = pb + ty + 4 * r;
    if (pr < P) out[(size_t)pr * KN + s0 + tx] = tile[tx][ty + 4 * r];
  }
}

// in [rows][cols] -> out [cols][out_rows], zeros in columns rows .. out_rows - 1
// of out.  64 x 64 tiles through LDS, 256-byte rows on both sides.
__global__ __launch_bounds__(256) void k_transpose32(const uint32_t *__restrict__ in,
                                                     uint32_t *__restrict__ out, uint32_t rows,
                                                     uint32_t cols, uint32_t out_rows) {
  __shared__ uint32_t tile[64][65];
  const uint32_t r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  const uint32_t tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
  for (uint32_t k = 0; k < 16; ++k) {
    const uint32_t r = r0 + ty + 4 * k, c = c0 + tx;
    tile[ty + 4 * k][tx] = r < rows && c < cols ? in[(size_t)r * cols + c] : 0u;
  }
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < 16; ++k) {
    const uint32_t c = c0 + ty + 4 * k, r = r0 + tx;
    if (c < cols && r < out_rows) out[(size_t)c * out_rows + r] = tile[tx][ty + 4 * k];
  }
}

// Timing data for the autotuner: word i = hash(i) & 0x0F7F7F7F (every byte a
// valid 7-bit limb, every word below 2^28).  Timing depends on the data: the
// matrix cores draw more power on random operands than on zeros.
__global__ void k_fill_tuning(uint32_t *__restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    uint32_t x = (uint32_t)i * 0x9E3779B1u ^ (uint32_t)(i >> 32);
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    p[i] = x & 0x0F7F7F7Fu;
  }
}

}  // namespace

hipError_t launch_fill_tuning(uint32_t *p, size_t n_words, hipStream_t s) {
  if (n_words == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n_words + 255) / 256, 65536);
  k_fill_tuning<<<(unsigned)blocks, 256, 0, s>>>(p, n_words);
  return hipGetLastError();
}

hipError_t launch_transpose32(const uint32_t *in, uint32_t *out, uint32_t rows, uint32_t cols,
                              uint32_t out_rows, hipStream_t s) {
  if (out_rows < rows || cols == 0 || out_rows == 0) return hipErrorInvalidValue;
  k_transpose32<<<dim3((out_rows + 63) / 64, (cols + 63) / 64), 256, 0, s>>>(in, out, rows, cols,
                                                                             out_rows);
  return hipGetLastError();
}

hipError_t launch_unpack_answers(const uint32_t *sm, uint32_t p_stride, uint32_t p0, uint32_t P,
                                 uint32_t KN, uint32_t *out, hipStream_t s) {
  if (KN % 64 != 0 || (size_t)p0 + P > p_stride) return hipErrorInvalidValue;
  if (P == 0) return hipSuccess;
  k_unpack_answers<<<dim3((P + 63) / 64, KN / 64), 256, 0, s>>>(sm, p_stride, p0, P, KN, out);
  return hipGetLastError();
}

hipError_t launch_pack_query_slot(const uint32_t *q_ntt, uint8_t *qatoms, uint32_t col_slot,
                                  uint32_t n_cb, uint32_t R, uint32_t N, uint32_t K,
                                  hipStream_t s) {
  if (2 * col_slot + 1 >= n_cb * kCB) return hipErrorInvalidValue;
  const uint32_t n_ib = r_pad(R) / kIB;
  const dim3 grid(N / 32, (n_ib + kPqIB - 1) / kPqIB, K);
  k_pack_query_slot<<<grid, 256, 0, s>>>(q_ntt, qatoms, col_slot, n_cb, R, N, K, n_ib);
  return hipGetLastError();
}

hipError_t launch_pack_db(const uint32_t *ntt_slab, uint8_t *atoms, uint32_t i0, uint32_t S,
                          uint32_t R, uint32_t C, uint32_t N, uint32_t K, hipStream_t s) {
  if (S % 32 != 0 || i0 % 32 != 0 || N % 32 != 0) return hipErrorInvalidValue;
  const uint32_t n_jb = c_pad(C) / kJB, n_ib = r_pad(R) / kIB;
  const dim3 grid(N / 32, n_jb, K * (S / 32));
  k_pack_db<<<grid, 256, 0, s>>>(ntt_slab, atoms, i0 / 32, S, C, N, n_jb, n_ib);
  return hipGetLastError();
}

hipError_t launch_read_db(const DbDesc &db, uint32_t i0, uint32_t ni, uint32_t j0, uint32_t nj,
                          uint32_t *out, hipStream_t s) {
  const size_t total = (size_t)ni * nj * db.K * db.N;
  if (total == 0) return hipSuccess;
  const size_t blocks = (total + 255) / 256;
  k_read_db<<<(unsigned)(blocks < 65536 ? blocks : 65536), 256, 0, s>>>(db, i0, ni, j0, nj, out);
  return hipGetLastError();
}

hipError_t launch_pack_query(const uint32_t *q_ntt, uint8_t *qatoms, uint32_t B, uint32_t R,
                             uint32_t N, uint32_t K, hipStream_t s) {
  const uint32_t n_ib = r_pad(R) / kIB, n_cb = (2 * B + kCB - 1) / kCB;
  const dim3 grid(N / 32, n_ib, K * n_cb);
  k_pack_query<<<grid, 256, 0, s>>>(q_ntt, qatoms, B, R, N, K, n_ib, n_cb);
  return hipGetLastError();
}

}  // namespace pir
