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
//  * k_scan_b1 / k_scan_b1r (B = 1): bandwidth-bound streaming.
//    v_mfma_i32_16x16x64_i8 with 4 database rows x 4 limbs per A operand and
//    the two ciphertext components x 4 limbs (half the B columns) per B
//    operand.  The block splits the slot's query limbs straight from the
//    NTT-form query into LDS; each wave streams its database atoms from HBM,
//    in groups of UNR k-blocks (k_scan_b1) or through a register ring that
//    never drains between row blocks (k_scan_b1r).
//  * k_scan_mfma (B > 1): v_mfma_i32_32x32x32_i8 over whole atoms.  A wave
//    owns JBW x 8 database rows and CBW x 8 query columns; database atoms come
//    through a register ring D contraction steps deep, query atoms through
//    LDS chunks shared by the block's four waves (three buffers filled by
//    LDS DMA, or two filled through staging registers).
#include <hip/hip_ext.h>

#include <algorithm>

#include "device_util.h"
#include "pir_internal.h"

namespace pir {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr uint32_t kB1Chunk = 64;  // query ibs split into LDS per chunk (16 KiB)

// Instruction-class masks of the scheduling-group builtin.
constexpr int kSgMfma = 0x008, kSgVmemRead = 0x020, kSgDsRead = 0x100, kSgDsWrite = 0x200;

// Scan launches take a table of up to kMaxFused jobs.  The grid is the
// concatenation of the jobs' blocks, each job's count rounded up to a
// multiple of 8 (job j owns grid blocks [first, first + round8(n_blocks))),
// so every job is spread evenly over the 8 XCDs; inside a job the blocks of
// one XCD take a contiguous run of the job's logical indices.  (One XCD-
// contiguous mapping over the whole concatenation would hand whole XCDs to
// one job, and jobs whose blocks cost different amounts would leave XCDs
// idle.)  A block finds its job by a uniform search of the table in the
// kernel-argument segment.
constexpr int kMaxFused = 8;

struct B1Job {
  DbDesc db;
  const uint32_t *q;  // NTT-form query [1][R][2][K][N]
  uint32_t *out;      // answer [1][C][2][K][N]
  uint32_t slot0, n_slots;  // slots scanned: [slot0, slot0 + n_slots)
  uint32_t jpb;       // jbs per block
  uint32_t n_blocks;  // blocks of this job
  uint32_t first;     // first grid block of this job (a multiple of 8)
};

struct B1Args {
  B1Job jobs[kMaxFused];
  uint32_t n_jobs, total;
};

template <typename Args>
__device__ __forceinline__ uint32_t find_job(const Args &a, uint32_t bid) {
  uint32_t jid = 0;
#pragma unroll
  for (int j = 1; j < kMaxFused; ++j)
    if ((uint32_t)j < a.n_jobs && bid >= a.jobs[j].first) jid = j;
  return jid;
}

// The logical index of grid block `bid` inside its job (see above); at or
// beyond the job's n_blocks the block is idle.
template <typename Job>
__device__ __forceinline__ uint32_t job_logical(const Job &a, uint32_t bid) {
  return xcd_logical(bid - a.first, (a.n_blocks + 7u) & ~7u);
}

// Reduce the lane's partial sum s over the 4 lanes b = 0..3 (lane bits 0,1)
// with quad permutes (DPP quad_perm [1,0,3,2] then [2,3,0,1]).
// Input s in [0, 2q); output in [0, q).
__device__ __forceinline__ uint32_t quad_sum_mod(uint32_t s, uint32_t q) {
  s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0xB1, 0xF, 0xF, false);  // < 4q
  s += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)s, 0x4E, 0xF, 0xF, false);  // < 8q
  s = csub(s, 4 * q);
  s = csub(s, 2 * q);
  return csub(s, q);
}

// x moved from the lane given by the quad permutation CTRL, 64 bits at a time.
// Every lane's source lies in its own quad, so no lane reads an invalid source
// and the plain move (no old value to preserve) is exact; it spares the
// register initialisation an update with an old value costs.
template <int CTRL>
__device__ __forceinline__ double quad_perm_f64(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One output of the batched scan from its 16 limb sums, in two stages.  This
// lane holds P[a] = acc[(row, a)][(col, b)] for a = 0..3 and its own b
// (wb = 2^(7b)); the other three lanes of the quad hold the other b.  The
// target is  sum_{a,b} P[a][b] * 2^(7(a+b))  mod q.  Everything runs in fp64 on
// exact integers:
//  * L = sum_a P[a] 2^(7a) < 2^29 * 2^21.01 < 2^51 (P[a] < 2^29 for R <= 32768);
//  * r = L - rint(L/q) q is exact (the product and the difference are integers
//    below 2^53) and |r| <= q/2 + 1;
//  * z = r * 2^(7b) summed over the quad is below 2^50 in magnitude, and every
//    lane of the quad ends with the same z (quad_partial);
//  * y = z - rint(z/q) q is exact with |y| <= q/2 + 1; adding q when y < 0
//    gives the canonical residue (quad_final).
// The quotient estimates only choose which multiple of q to subtract, so
// their rounding never affects the result.
__device__ __forceinline__ double quad_partial(int p0, int p1, int p2, int p3, double wb,
                                               double qd, double inv_q) {
  const double L = (double)p0 + 128.0 * (double)p1 + 16384.0 * (double)p2 + 2097152.0 * (double)p3;
  const double r = L - __builtin_rint(L * inv_q) * qd;
  double z = r * wb;
  z += quad_perm_f64<0xB1>(z);
  z += quad_perm_f64<0x4E>(z);
  return z;
}

__device__ __forceinline__ uint32_t quad_final(double z, double qd, double inv_q, uint32_t q) {
  const int y = (int)(z - __builtin_rint(z * inv_q) * qd);
  return (uint32_t)(y < 0 ? y + (int)q : y);
}

// sum_a P[a] * 2^(7a) mod q for the four limb sums P[a] < 2^31 of one lane.
// The sum T is exact in 64 bits (< 2^53) and exactly representable as a
// double, so a double quotient estimate is off by at most one; the int32
// remainder T - qhat*q then lies in (-q, 2q) and two corrections make it exact.
__device__ __forceinline__ uint32_t limb_sum_mod(uint32_t p0, uint32_t p1, uint32_t p2, uint32_t p3,
                                                 uint32_t q, double inv_q) {
  const uint64_t T = (uint64_t)p0 + ((uint64_t)p1 << 7) + ((uint64_t)p2 << 14) +
                     ((uint64_t)p3 << 21);
  const uint32_t qhat = (uint32_t)((double)T * inv_q);
  int32_t r = (int32_t)((uint32_t)T - qhat * q);
  r += r < 0 ? (int32_t)q : 0;
  r -= r >= (int32_t)q ? (int32_t)q : 0;
  return (uint32_t)r;
}

template <bool NT>
__device__ __forceinline__ v4i load_atom16(const uint8_t *p) {
  const v4i *v = reinterpret_cast<const v4i *>(p);
  if constexpr (NT) {
    return __builtin_nontemporal_load(v);
  } else {
    return *v;
  }
}

// Split the slot's query residues of atoms ib0 .. ib0 + nib - 1 into limb bytes
// in LDS: item (ibl, half, c, e4) covers i = 32 (ib0+ibl) + 16 half + 4 e4 + u,
// u < 4, and writes one word per limb b at LDS lane (half, 4c + b), bytes
// 4 e4 .. 4 e4 + 3.  Rows past R read as zero.
__device__ __forceinline__ void b1_split_query(uint32_t *sq, const uint32_t *qbase, size_t qrow,
                                               uint32_t R, uint32_t ib0, uint32_t nib,
                                               uint32_t tid) {
  for (uint32_t idx = tid; idx < nib * 16; idx += 256) {
    const uint32_t ibl = idx >> 4, r = idx & 15;
    const uint32_t half = r >> 3, c = (r >> 2) & 1, e4 = r & 3;
    const uint32_t i0 = (ib0 + ibl) * 32 + half * 16 + e4 * 4;
    uint32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = (i0 + u < R) ? qbase[((size_t)(i0 + u) * 2 + c) * qrow] : 0u;
#pragma unroll
    for (uint32_t b = 0; b < 4; ++b) {
      uint32_t w = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) w |= ((v[u] >> (7 * b)) & 127u) << (8 * u);
      sq[((ibl * 2 + half) * 8 + c * 4 + b) * 4 + e4] = w;
    }
  }
}

// Epilogue of both batch-1 kernels for row block jb.  Lane holds rows
// 4*(lane>>4) + r (row = 4 jl' + a, a = r) of column lane & 15 (= 4 cc + b).
__device__ __forceinline__ void b1_epilogue(const v4i (&acc)[2], uint32_t jb, uint32_t lane,
                                            const DbDesc &db, const DevPrime &P, uint32_t k,
                                            uint32_t t, uint32_t *out) {
  const uint32_t b = lane & 3, cc = (lane >> 2) & 3, jlp = lane >> 4;
  const uint32_t q = P.q, wb = P.w[b], wbsh = P.w_sh[b];
  const double inv_q = 1.0 / (double)q;
  const size_t KN = (size_t)db.K * db.N;
#pragma unroll
  for (int jh = 0; jh < 2; ++jh) {
    const v4i &A = acc[jh];
    const uint32_t u = limb_sum_mod(A[0], A[1], A[2], A[3], q, inv_q);
    const uint32_t s = quad_sum_mod(mul_shoup(u, wb, wbsh, q), q);
    const uint32_t j = jb * 8 + jh * 4 + jlp;
    if (b == 0 && cc < 2 && j < db.C) out[((size_t)j * 2 + cc) * KN + (size_t)k * db.N + t] = s;
  }
}

template <int JBW, int UNR, bool NT>
__global__ __launch_bounds__(256) void k_scan_b1(const B1Args args) {
  __shared__ uint32_t sq[kB1Chunk * 64];
  if (blockIdx.x >= args.total) return;
  const B1Job &a = args.jobs[find_job(args, blockIdx.x)];
  const uint32_t L = job_logical(a, blockIdx.x);
  if (L >= a.n_blocks) return;
  const DbDesc &db = a.db;
  const uint32_t slot = a.slot0 + L % a.n_slots, jchunk = L / a.n_slots;
  const uint32_t k = slot >> db.log2n, t = slot & (db.N - 1);
  const DevPrime &P = db.primes[k];

  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint32_t g = lane >> 4, m = lane & 15;
  const uint32_t n_ib = db.n_ib, n_jb = db.n_jb;
  const uint32_t jb_begin = jchunk * a.jpb;
  const uint32_t jb_end = min(jb_begin + a.jpb, n_jb);
  const uint8_t *slot_atoms = db.atoms + (size_t)slot * n_jb * n_ib * kAtomBytes;
  const uint32_t lane_off = (g >> 1) * 1024 + (g & 1) * 512 + m * 16;
  const bool bzero = m >= 8;
  const size_t qrow = (size_t)db.K * db.N;  // stride between (i, c) rows of the query
  const uint32_t *qbase = a.q + (size_t)k * db.N + t;
  const uint4 *sq4 = reinterpret_cast<const uint4 *>(sq);

  v4i acc[JBW][2];
#pragma unroll
  for (int w = 0; w < JBW; ++w) acc[w][0] = acc[w][1] = v4i{0, 0, 0, 0};

  for (uint32_t ib0 = 0; ib0 < n_ib; ib0 += kB1Chunk) {
    const uint32_t nib = min(kB1Chunk, n_ib - ib0);  // even: R_pad is a multiple of 64
    __syncthreads();
    b1_split_query(sq, qbase, qrow, db.R, ib0, nib, tid);
    __syncthreads();
    const uint32_t nkb = nib >> 1;
#pragma unroll
    for (int w = 0; w < JBW; ++w) {
      const uint32_t jb = jb_begin + wave + 4 * w;
      if (jb >= jb_end) break;
      const uint8_t *base = slot_atoms + ((size_t)jb * n_ib + ib0) * kAtomBytes + lane_off;
      auto mma = [&](const v4i &x0, const v4i &x1, uint32_t kb) {
        // every lane reads a valid address; lanes of the empty columns 8..15 then zero it
        const uint4 x = sq4[(2 * kb + (g >> 1)) * 16 + (g & 1) * 8 + (m & 7)];
        const v4i bv = bzero ? v4i{0, 0, 0, 0} : v4i{(int)x.x, (int)x.y, (int)x.z, (int)x.w};
        acc[w][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(x0, bv, acc[w][0], 0, 0, 0);
        acc[w][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(x1, bv, acc[w][1], 0, 0, 0);
      };
      uint32_t kb0 = 0;
      // full groups: UNR k-blocks of loads issued before the first of their MFMAs
      for (; kb0 + UNR <= nkb; kb0 += UNR) {
        v4i a0[UNR], a1[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          a0[u] = load_atom16<NT>(base + (size_t)(kb0 + u) * 2048);
          a1[u] = load_atom16<NT>(base + (size_t)(kb0 + u) * 2048 + 256);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) mma(a0[u], a1[u], kb0 + u);
      }
      for (; kb0 < nkb; ++kb0) {
        const v4i x0 = load_atom16<NT>(base + (size_t)kb0 * 2048);
        const v4i x1 = load_atom16<NT>(base + (size_t)kb0 * 2048 + 256);
        mma(x0, x1, kb0);
      }
    }
  }

#pragma unroll
  for (int w = 0; w < JBW; ++w) {
    const uint32_t jb = jb_begin + wave + 4 * w;
    if (jb >= jb_end) break;
    b1_epilogue(acc[w], jb, lane, db, P, k, t, a.out);
  }
}

// Batch-1 scan with a continuous load stream.  Each wave walks its row blocks
// w = 0 .. nw-1 and, within each, the k-blocks of the current query chunk as
// one sequence through a register ring D k-blocks deep: the MFMAs of k-block
// s are followed by the loads of k-block s + D.  In the last D k-blocks of a
// row those loads come from the next row block, or from the next chunk's first
// row block, so the loads in flight never drain between rows; the first row's
// ring is requested before the query split.  Scheduling groups keep the
// order LDS read, two MFMAs, two loads per k-block.  Needs every chunk's
// k-block count to be a multiple of D (the launcher checks).
template <int JBW, int D, bool NT>
__global__ __launch_bounds__(256) void k_scan_b1r(const B1Args args) {
  __shared__ uint32_t sq[kB1Chunk * 64];
  if (blockIdx.x >= args.total) return;
  const B1Job &a = args.jobs[find_job(args, blockIdx.x)];
  const uint32_t L = job_logical(a, blockIdx.x);
  if (L >= a.n_blocks) return;
  const DbDesc &db = a.db;
  const uint32_t slot = a.slot0 + L % a.n_slots, jchunk = L / a.n_slots;
  const uint32_t k = slot >> db.log2n, t = slot & (db.N - 1);
  const DevPrime &P = db.primes[k];
  const uint32_t q = P.q;

  const uint32_t tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const uint32_t g = lane >> 4, m = lane & 15;
  const uint32_t n_ib = db.n_ib, n_jb = db.n_jb;
  const uint32_t jb_begin = jchunk * a.jpb;
  const uint32_t jb_end = min(jb_begin + a.jpb, n_jb);
  // row blocks of this wave: jb_begin + wave + 4 w for w < nw
  const uint32_t nw = jb_begin + wave < jb_end ? min((uint32_t)JBW, (jb_end - jb_begin - wave + 3) / 4) : 0;
  const uint8_t *slot_atoms = db.atoms + (size_t)slot * n_jb * n_ib * kAtomBytes;
  const uint32_t lane_off = (g >> 1) * 1024 + (g & 1) * 512 + m * 16;
  const bool bzero = m >= 8;
  const size_t qrow = (size_t)db.K * db.N;
  const uint32_t *qbase = a.q + (size_t)k * db.N + t;
  const uint4 *sq4 = reinterpret_cast<const uint4 *>(sq);
  auto row_ptr = [&](uint32_t w, uint32_t ib0) {
    return slot_atoms + ((size_t)(jb_begin + wave + 4 * w) * n_ib + ib0) * kAtomBytes + lane_off;
  };

  v4i acc[JBW][2];
#pragma unroll
  for (int w = 0; w < JBW; ++w) acc[w][0] = acc[w][1] = v4i{0, 0, 0, 0};
  v4i r0[D], r1[D];
  if (nw > 0) {
    const uint8_t *p = row_ptr(0, 0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      r0[d] = load_atom16<NT>(p + (size_t)d * 2048);
      r1[d] = load_atom16<NT>(p + (size_t)d * 2048 + 256);
    }
  }

  for (uint32_t ib0 = 0; ib0 < n_ib; ib0 += kB1Chunk) {
    const uint32_t nib = min(kB1Chunk, n_ib - ib0);
    const uint32_t nkb = nib >> 1, ib_next = ib0 + kB1Chunk;
    __syncthreads();
    b1_split_query(sq, qbase, qrow, db.R, ib0, nib, tid);
    __syncthreads();
#pragma unroll
    for (int w = 0; w < JBW; ++w) {
      if ((uint32_t)w < nw) {
        auto mma = [&](const v4i &x0, const v4i &x1, uint32_t kb) {
          const uint4 x = sq4[(2 * kb + (g >> 1)) * 16 + (g & 1) * 8 + (m & 7)];
          const v4i bv = bzero ? v4i{0, 0, 0, 0} : v4i{(int)x.x, (int)x.y, (int)x.z, (int)x.w};
          acc[w][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(x0, bv, acc[w][0], 0, 0, 0);
          acc[w][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(x1, bv, acc[w][1], 0, 0, 0);
        };
        const uint8_t *base = row_ptr(w, ib0);
        uint32_t kb0 = 0;
        for (; kb0 + D < nkb; kb0 += D) {
#pragma unroll
          for (int d = 0; d < D; ++d) {
            mma(r0[d], r1[d], kb0 + d);
            r0[d] = load_atom16<NT>(base + (size_t)(kb0 + D + d) * 2048);
            r1[d] = load_atom16<NT>(base + (size_t)(kb0 + D + d) * 2048 + 256);
          }
#pragma unroll
          for (int d = 0; d < D; ++d) {
            __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
            __builtin_amdgcn_sched_group_barrier(kSgMfma, 2, 0);
            __builtin_amdgcn_sched_group_barrier(kSgVmemRead, 2, 0);
          }
        }
        // last D k-blocks of the row: refill from the next row, else from the
        // next chunk's first row, else not at all
        const bool more_row = (uint32_t)w + 1 < nw;
        if (more_row || ib_next < n_ib) {
          const uint8_t *nb = more_row ? row_ptr(w + 1, ib0) : row_ptr(0, ib_next);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            mma(r0[d], r1[d], kb0 + d);
            r0[d] = load_atom16<NT>(nb + (size_t)d * 2048);
            r1[d] = load_atom16<NT>(nb + (size_t)d * 2048 + 256);
          }
#pragma unroll
          for (int d = 0; d < D; ++d) {
            __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
            __builtin_amdgcn_sched_group_barrier(kSgMfma, 2, 0);
            __builtin_amdgcn_sched_group_barrier(kSgVmemRead, 2, 0);
          }
        } else {
#pragma unroll
          for (int d = 0; d < D; ++d) mma(r0[d], r1[d], kb0 + d);
        }
      }
    }
  }

#pragma unroll
  for (int w = 0; w < JBW; ++w)
    if ((uint32_t)w < nw) b1_epilogue(acc[w], jb_begin + wave + 4 * w, lane, db, P, k, t, a.out);
}

// ---------------------------------------------------------------------------
constexpr uint32_t kKCB = 4;  // contraction steps per staged query chunk

struct MfJob {
  DbDesc db;
  const uint8_t *qatoms;  // query atoms [K][N][n_ib][cb_stride] or [K][N][cb_stride][n_ib]
  uint32_t *out;          // answers, slot-major: [K N][p_stride]
  uint32_t B, n_cb, cb_stride, p_stride;
  uint32_t q_ibs, q_cbs;  // atoms between consecutive ib, and between consecutive cb
  uint32_t slot0, n_jg, n_cbt;  // work item = (slot, row group, column tile)
  uint32_t n_items, n_blocks;   // items; blocks (block L takes items L, L + n_blocks, ...)
  uint32_t first;               // first logical block of this job
};

struct MfArgs {
  MfJob jobs[kMaxFused];
  uint32_t n_jobs, total;
};

// Third descriptor word of a raw (unformatted, stride 0) buffer resource.
constexpr int kBufferWord3 = 0x00020000;


// Where one work item's operands live, as seen by one wave.
template <int JBW>
struct MfItem {
  uint32_t slot, cb0, ncb;
  uint32_t jbs[JBW];
  bool jv[JBW];
  const uint8_t *rows[JBW];      // first database atom of each row block (wave-uniform)
  __amdgpu_buffer_rsrc_t qrs;    // the slot's query atoms
};

template <int JBW, int CBW, int NW>
__device__ __forceinline__ void mf_item(const MfJob &a, uint32_t it, uint32_t wave,
                                        MfItem<JBW> &m) {
  const DbDesc &db = a.db;
  // column tiles of the same rows are adjacent, then row groups of one slot
  const uint32_t cbt = it % a.n_cbt, rest = it / a.n_cbt;
  const uint32_t jg = rest % a.n_jg;
  m.slot = a.slot0 + rest / a.n_jg;
  m.cb0 = cbt * CBW;
  m.ncb = min((uint32_t)CBW, a.n_cb - m.cb0);
#pragma unroll
  for (int w = 0; w < JBW; ++w) {
    m.jbs[w] = (jg * NW + wave) * JBW + w;
    m.jv[w] = m.jbs[w] < db.n_jb;
    // rows past C read row block 0: valid memory, results discarded
    m.rows[w] = db.atoms +
                ((size_t)m.slot * db.n_jb + (m.jv[w] ? m.jbs[w] : 0)) * db.n_ib * kAtomBytes;
  }
  // A raw buffer resource over the slot's query atoms: a load whose offset is
  // past the resource's size returns zeros, so staging needs no branch.
  const uint32_t q_bytes = db.n_ib * a.cb_stride * kAtomBytes;
  m.qrs = __builtin_amdgcn_make_buffer_rsrc((void *)(a.qatoms + (size_t)m.slot * q_bytes), (short)0,
                                            (int)q_bytes, kBufferWord3);
}

// A block is NW waves (four: one per SIMD; eight: two per SIMD sharing one
// query chunk); wave w owns row blocks (NW jg + w) JBW .. + JBW - 1 and CBW
// query column blocks of one work item (slot, jg, column tile).  Blocks
// are persistent over a strided sequence of items (L, L + n_blocks, ...), so
// blocks running at the same time work on neighbouring items and share the
// slot's query atoms in L2.  The contraction of an item runs over S steps
// (one 32-row atom each, n_ib rounded up to D; steps past n_ib read valid
// memory and meet zero query atoms).
//
// Pipeline, per wave:
//  * database atoms: a register ring D steps deep; the atom of step s + D is
//    requested right after the MFMAs of step s have read ring slot s mod D.
//    Near the end of an item the ring fills with the next item's first steps,
//    so the epilogue runs while they are in flight;
//  * query atoms: LDS chunks of kKCB steps.  Chunk n + 1 is published by a
//    barrier one step before chunk n ends (with one-step B prefetch; at its
//    last step without).  With LDS DMA (three buffers) the loads of chunk
//    n + 3 (of this item or the next) go out right after that barrier, into
//    the buffer chunk n used, about two chunks ahead of their use, the same
//    lead as the ring's; with register staging (two buffers) the loads of
//    chunk n + 2 go out there and are written to LDS one step before the
//    next barrier;
//  * the order inside a step is pinned with scheduling groups, so the
//    compiler cannot sink the prefetches next to their uses.
// NTR selects the ring's cache policy: nontemporal when a launch has one
// column tile (no block reads a database atom twice), plain otherwise, so that
// the blocks of the other column tiles of the same rows, which run at about
// the same time on the same XCD, find the atoms in L2 (4 GiB-raw database,
// B = 128: HBM reads 104 -> 79 GB per launch).
// Every staging condition is wave-uniform, so no load sits under a divergent
// branch and the memory counters stay exact.
// One 16-byte-per-lane load from a raw buffer straight into LDS (the 64 lanes
// fill lds .. lds + 1023).  Issued from inline assembly, so the compiler's
// wait-count bookkeeping does not see it: every wait for these loads is
// explicit, and the compiler's own waits for other loads stay correct because
// vector-memory loads complete in issue order (an unseen newer load can only
// make a wait longer).
__device__ __forceinline__ void lds_dma_b128(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t lds) {
  asm volatile("buffer_load_dwordx4 %0, %1, 0 offen lds" ::"v"(off), "s"(rs), "{m0}"(lds) : "memory");
}

template <int JBW, int CBW, int D, int OCC, int NW, bool NTR>
__global__ __launch_bounds__(64 * NW, OCC) void k_scan_mfma(const MfArgs args) {
  static_assert(D % kKCB == 0 && kKCB >= 2, "ring depth must be a multiple of the query chunk");
  constexpr uint32_t kAtoms = kKCB * CBW;      // query atoms per chunk
  constexpr uint32_t kBuf = kAtoms * 64;       // uint4 per LDS buffer
  constexpr uint32_t kPer = (kAtoms + NW - 1) / NW;  // chunk atoms per wave
  constexpr int kWps = NW / 4 * OCC;                  // waves per SIMD
  constexpr int kM = JBW * CBW;                // MFMAs per step
  // Query chunks go straight to LDS through three buffers when they fit
  // (160 KiB of LDS per CU), else through staging registers and two buffers.
  constexpr bool kDma = 3 * kBuf * 16 * OCC <= 160 * 1024;
  static_assert(kAtoms % NW == 0, "every wave stages the same number of atoms");
  __shared__ uint4 sq[(kDma ? 3 : 2) * kBuf];
  if (blockIdx.x >= args.total) return;
  const MfJob &a = args.jobs[find_job(args, blockIdx.x)];
  const uint32_t L = job_logical(a, blockIdx.x);
  if (L >= a.n_blocks) return;
  const DbDesc &db = a.db;
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t n_ib = db.n_ib, q_ibs = a.q_ibs, q_cbs = a.q_cbs;
  // Steps per item: n_ib rounded up to the ring depth, and at least as many
  // chunks as the staging looks ahead (two, three with LDS DMA), so that it
  // never reaches past the next item.  Extra steps meet zero query atoms; their
  // database reads run at most S - n_ib atoms past the last row block of the
  // last slot, which the launcher checks against the database's tail padding.
  const uint32_t S = (max(n_ib, (kDma ? 3 : 2) * kKCB) + D - 1) / D * D;
  const uint32_t nc = S / kKCB;  // chunks per item
  const uint32_t lane_off = lane * 16;

  uint32_t it = L;
  MfItem<JBW> cur, nxt;
  mf_item<JBW, CBW, NW>(a, it, wave, cur);
  bool has_next = it + a.n_blocks < a.n_items;
  if (has_next) mf_item<JBW, CBW, NW>(a, it + a.n_blocks, wave, nxt);
  else nxt = cur;

  // atom of step ks (< S + D) of row block w: this item, else the next item's
  // step ks - S, else (last item) this item's step 0
  auto ring_ptr = [&](int w, uint32_t ks) {
    const uint8_t *p = ks < S ? cur.rows[w] + (size_t)ks * kAtomBytes
                              : has_next ? nxt.rows[w] + (size_t)(ks - S) * kAtomBytes : cur.rows[w];
    return reinterpret_cast<const v4i *>(p + lane_off);
  };
  auto ring_load = [](const v4i *p) {
    if constexpr (NTR) {
      return __builtin_nontemporal_load(p);
    } else {
      return *p;
    }
  };
  // query atoms of chunk n (< nc + 2) counted from this item's first: atom
  // (kk, c) of a chunk goes to wave (kk CBW + c) mod NW; zero past n_ib, past
  // the batch's column blocks and past the last item
  auto stage_load = [&](uint32_t n, v4i (&st)[kPer]) {
    const bool mine = n < nc;
    const uint32_t ln = mine ? n : n - nc;
    const bool live = mine || has_next;
    const uint32_t cb0 = mine ? cur.cb0 : nxt.cb0, ncb = mine ? cur.ncb : nxt.ncb;
    const __amdgpu_buffer_rsrc_t rs = mine ? cur.qrs : nxt.qrs;
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
      const uint32_t ai = wave + NW * r;
      const uint32_t kk = ai / CBW, c = ai % CBW, ks = ln * kKCB + kk;
      const bool ok = live && (kAtoms % NW == 0 || ai < kAtoms) && ks < n_ib && c < ncb;
      // offsets are below 2^26; setting bit 31 puts a dead load past the
      // resource's end (zeros) without a branch
      const uint32_t off = (((ks * q_ibs + (cb0 + c) * q_cbs) * 64 + lane) * 16) | ((uint32_t)!ok << 31);
      st[r] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    }
  };
  auto stage_store = [&](uint4 *buf, const v4i (&st)[kPer]) {
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
      const uint32_t ai = wave + NW * r;
      if (kAtoms % NW == 0 || ai < kAtoms)
        buf[ai * 64 + lane] = make_uint4(st[r].x, st[r].y, st[r].z, st[r].w);
    }
  };
  // LDS DMA of chunk n into buffer bi, same atoms and zeros as stage_load
  auto stage_dma = [&](uint32_t n, uint32_t bi) {
    const bool mine = n < nc;
    const uint32_t ln = mine ? n : n - nc;
    const bool live = mine || has_next;
    const uint32_t cb0 = mine ? cur.cb0 : nxt.cb0, ncb = mine ? cur.ncb : nxt.ncb;
    const __amdgpu_buffer_rsrc_t rs = mine ? cur.qrs : nxt.qrs;
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
      const uint32_t ai = wave + NW * r;
      const uint32_t kk = ai / CBW, c = ai % CBW, ks = ln * kKCB + kk;
      const bool ok = live && ks < n_ib && c < ncb;
      const uint32_t off = (((ks * q_ibs + (cb0 + c) * q_cbs) * 64 + lane) * 16) | ((uint32_t)!ok << 31);
      const uint32_t lds = (uint32_t)(size_t)(sq + (bi * kAtoms + ai) * 64);
      lds_dma_b128(rs, off, __builtin_amdgcn_readfirstlane(lds));
    }
  };
  auto b_read = [&](const uint4 *src, v4i (&bv)[CBW]) {
#pragma unroll
    for (int c = 0; c < CBW; ++c) {
      const uint4 u = src[c * 64 + lane];
      bv[c] = v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
    }
  };

  constexpr bool kPf = kWps == 1 || JBW * D * 4 + CBW * 8 <= 64;
  // LDS DMA: chunk n + 3 is requested right after the barrier that publishes
  // chunk n + 1, into the buffer chunk n used, and waited for at the barrier
  // that publishes it.  By then this wave has issued, after it, the ring loads
  // of two chunks' steps and the next chunk's requests (fewer in the first
  // chunks); kVmWait is the smallest of these counts.
  constexpr uint32_t kSpan = D + kKCB - (kPf ? 1 : 0) < 2 * kKCB ? D + kKCB - (kPf ? 1 : 0) : 2 * kKCB;
  constexpr uint32_t kVmWait = kPer + JBW * kSpan;
  static_assert(!kDma || 2 * kPer + D * JBW < 64, "wait counts fit the vmcnt field");
  v4i ring[D][JBW];
  v4i st[kPer];  // staging registers (register staging only)
  if (kDma) {
    stage_dma(0, 0);
    stage_dma(1, 1);
    stage_dma(2, 2);
  }
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int w = 0; w < JBW; ++w) ring[d][w] = ring_load(ring_ptr(w, d));
  if (kDma) {
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(2 * kPer + D * JBW) : "memory");
  } else {
    stage_load(0, st);
    stage_store(sq, st);
    stage_load(1, st);
    __syncthreads();
  }
  // Normally the B operands of step s + 1 are read during step s.  Two waves
  // per SIMD with a deep ring have no registers for a second set: each step
  // then reads its own B operands first and the other wave's MFMAs cover the
  // LDS latency.
  // Step of a chunk that publishes the next chunk.  The buffer it overwrites
  // was last read for the previous chunk's final step; that read comes before
  // the previous chunk's publishing barrier only if it is a prefetch (issued
  // one step early), so without prefetch the publish waits for the final step.
  constexpr int kPub = kPf ? (int)kKCB - 2 : (int)kKCB - 1;
  // MFMAs issued ahead of a publishing barrier (one wave per SIMD only: their
  // pin keeps the accumulators in AGPRs, which two waves per SIMD cannot afford)
  constexpr int kPre = kWps > 1 ? 0 : kM < 2 ? kM : 2;
  v4i bcur[CBW], bnext[CBW];
  if (kPf) b_read(sq, bcur);

  const uint32_t ncol = 2 * a.B;
  uint32_t chunk = 0;  // chunks completed by this block (LDS buffer parity)
  uint32_t b3 = 0;     // chunk mod 3 (LDS DMA buffer)
  for (;;) {
    v16i acc[JBW][CBW];
#pragma unroll
    for (int w = 0; w < JBW; ++w)
#pragma unroll
      for (int c = 0; c < CBW; ++c) acc[w][c] = v16i{};
    uint32_t cl = 0;  // chunk within the item
    for (uint32_t ks0 = 0; ks0 < S; ks0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int kk = d % (int)kKCB;
        const uint32_t bc = kDma ? b3 : chunk & 1;
        const uint32_t bn = kDma ? (b3 == 2 ? 0 : b3 + 1) : (chunk + 1) & 1;
        const uint4 *bcur_buf = sq + bc * kBuf;
        const uint4 *bnxt_buf = sq + bn * kBuf;
        // MFMAs of tiles [i0, i1) of this step (tile i = row block i / CBW,
        // column block i % CBW)
        auto mfmas = [&](int i0, int i1) {
#pragma unroll
          for (int i = i0; i < i1; ++i)
            acc[i / CBW][i % CBW] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                ring[d][i / CBW], bcur[i % CBW], acc[i / CBW][i % CBW], 0, 0, 0);
        };
        if (kPf && kk == (int)kKCB - 1) {
          // The chunk published last step becomes visible at a barrier taken
          // behind this step's first kPre MFMAs (they keep the matrix pipe busy
          // while the waves meet); then the next chunk's staging loads, then the
          // B operands of the next step from the new chunk.
          mfmas(0, kPre);
          // pin them ahead of the barrier (the MFMA builtin touches no memory,
          // so nothing else keeps the compiler from sinking it past)
#pragma unroll
          for (int i = 0; i < kPre; ++i) asm volatile("" : "+a"(acc[i / CBW][i % CBW]));
          if (kDma) {
            // every LDS read of this wave is done (the MFMAs above consumed
            // them), so buffer bc is free once all waves pass the barrier
            asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(kVmWait) : "memory");
            stage_dma(cl + 3, bc);
          } else {
            __syncthreads();
            stage_load(cl + 2, st);
          }
          __builtin_amdgcn_sched_barrier(0);
          b_read(bnxt_buf, bnext);
          mfmas(kPre, kM);
#pragma unroll
          for (int i = kPre; i < kM; ++i) {
            __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 0);
            if (i - kPre < CBW) __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
          }
        } else if (kPf) {
          // B operands of the next step (this chunk)
          b_read(bcur_buf + (kk + 1) * CBW * 64, bnext);
          mfmas(0, kM);
          if (!kDma && kk == kPub) {
            // publish chunk + 1: the staging stores ride between this step's
            // MFMAs, after its next-step B reads
            stage_store(sq + ((chunk + 1) & 1) * kBuf, st);
          }
#pragma unroll
          for (int i = 0; i < kM; ++i) {
            __builtin_amdgcn_sched_group_barrier(kSgMfma, 1, 0);
            if (i < CBW) __builtin_amdgcn_sched_group_barrier(kSgDsRead, 1, 0);
            else if (!kDma && kk == kPub && i - CBW < (int)kPer)
              __builtin_amdgcn_sched_group_barrier(kSgDsWrite, 1, 0);
          }
        } else {
          b_read(bcur_buf + kk * CBW * 64, bcur);
          mfmas(0, kM);
          __builtin_amdgcn_sched_group_barrier(kSgDsRead, CBW, 0);
          __builtin_amdgcn_sched_group_barrier(kSgMfma, kM, 0);
        }
#pragma unroll
        for (int w = 0; w < JBW; ++w)
          ring[d][w] = ring_load(ring_ptr(w, ks0 + D + d));
        __builtin_amdgcn_sched_group_barrier(kSgVmemRead, JBW, 0);
        if (!kPf && kk == kPub) {
          if (kDma) {
            // publish chunk + 1 after this step's reads and ring loads
            __builtin_amdgcn_sched_barrier(0);
            asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(kVmWait) : "memory");
            stage_dma(cl + 3, bc);
            __builtin_amdgcn_sched_barrier(0);
          } else {
            // publish chunk + 1 (after this step's ring loads), then fetch
            // chunk + 2 into the staging registers
            __builtin_amdgcn_sched_group_barrier(kSgDsWrite, kPer, 0);
            stage_store(sq + ((chunk + 1) & 1) * kBuf, st);
            __syncthreads();
            stage_load(cl + 2, st);
            // keep the staging loads here, a chunk ahead of their use
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        if (kk == (int)kKCB - 1) ++chunk, ++cl, b3 = b3 == 2 ? 0 : b3 + 1;
        if (kPf) {
#pragma unroll
          for (int c = 0; c < CBW; ++c) bcur[c] = bnext[c];
        }
      }
    }
    // Epilogue of the item.  32x32 result: lane holds column lane & 31
    // (= 4 cc + b) and, in register r, row 8 (r >> 2) + 4 (lane >> 5) + (r & 3)
    // (row = 4 jl + a), so the four registers 4 qq .. 4 qq + 3 of a lane are
    // the limbs a = 0..3 of one (row, column, b) and the four lanes b = 0..3 of
    // a quad complete the output.
    {
      const uint32_t b = lane & 3, cc = (lane >> 2) & 7, hi = lane >> 5;
      const uint32_t q = db.primes[cur.slot >> db.log2n].q;
      const double qd = (double)q, inv_q = 1.0 / qd, wb = (double)(1u << (7 * b));
      // After quad_partial the four lanes of a quad agree; lane b finishes and
      // stores the output of register group qq = b, i.e. row 8 jb + 2 b + hi.
      // Answer polynomial p = (query C + j) 2 + component with query = col / 2
      // and component = col % 2: in one store the 16 lanes of a query write 16
      // consecutive words (8 rows x 2 components) of the slot's row.
      const uint32_t jrow = 2 * b + hi;
      uint32_t *out_lane = a.out + (size_t)cur.slot * a.p_stride +
                           ((size_t)(cur.cb0 * 4 + (cc >> 1)) * db.C + jrow) * 2 + (cc & 1);
#pragma unroll
      for (int w = 0; w < JBW; ++w) {
#pragma unroll
        for (int c = 0; c < CBW; ++c) {
          double z[4];
#pragma unroll
          for (int qq = 0; qq < 4; ++qq)
            z[qq] = quad_partial(acc[w][c][4 * qq], acc[w][c][4 * qq + 1], acc[w][c][4 * qq + 2],
                                 acc[w][c][4 * qq + 3], wb, qd, inv_q);
          const double zb = b == 0 ? z[0] : b == 1 ? z[1] : b == 2 ? z[2] : z[3];
          const uint32_t mine = quad_final(zb, qd, inv_q, q);
          const uint32_t col = (cur.cb0 + c) * 8 + cc, j = cur.jbs[w] * 8 + jrow;
          if (cur.jv[w] && (uint32_t)c < cur.ncb && j < db.C && col < ncol)
            out_lane[((size_t)c * 4 * db.C + (size_t)cur.jbs[w] * 8) * 2] = mine;
        }
      }
    }
    if (!has_next) break;
    // the ring, the published chunk and the staged chunks already hold the
    // next item's first steps
    it += a.n_blocks;
    cur = nxt;
    has_next = it + a.n_blocks < a.n_items;
    if (has_next) mf_item<JBW, CBW, NW>(a, it + a.n_blocks, wave, nxt);
  }
  // LDS DMA requests past the last chunk are still in flight: the wave may
  // not end before they have written this workgroup's LDS
  if (kDma) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

inline uint32_t round8(uint32_t x) { return (x + 7) / 8 * 8; }

// Launchers take optional events that the launch itself records at the
// kernel's start and end (no separate marker commands on the stream).
template <int JBW, int UNR, bool NT>
hipError_t run_b1(const ScanJob *jobs, size_t n, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  B1Args a{};
  uint32_t total = 0;
  for (size_t i = 0; i < n; ++i) {
    const ScanJob &job = jobs[i];
    B1Job &b = a.jobs[i];
    b.db = job.db;
    b.q = job.q_ntt;
    b.out = job.out;
    b.slot0 = job.slot0;
    b.n_slots = job.n_slots;
    b.jpb = 4 * JBW;
    b.n_blocks = b.n_slots * ((job.db.n_jb + b.jpb - 1) / b.jpb);
    b.first = total;
    total += round8(b.n_blocks);
  }
  a.n_jobs = (uint32_t)n;
  a.total = total;
  if (total == 0) return hipSuccess;
  hipExtLaunchKernelGGL(k_scan_b1<JBW, UNR, NT>, dim3(total), dim3(256), 0, s, e0, e1, 0, a);
  return hipGetLastError();
}

// The ring kernel when every query chunk's k-block count (kB1Chunk / 2, and
// half the last chunk's atoms) is a multiple of D; else the grouped kernel.
template <int JBW, int D, bool NT>
hipError_t run_b1r(const ScanJob *jobs, size_t n, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  for (size_t i = 0; i < n; ++i) {
    const uint32_t tail = jobs[i].db.n_ib % kB1Chunk;
    if ((kB1Chunk / 2) % D != 0 || (tail / 2) % D != 0) return run_b1<JBW, D, NT>(jobs, n, s, e0, e1);
  }
  B1Args a{};
  uint32_t total = 0;
  for (size_t i = 0; i < n; ++i) {
    const ScanJob &job = jobs[i];
    B1Job &b = a.jobs[i];
    b.db = job.db;
    b.q = job.q_ntt;
    b.out = job.out;
    b.slot0 = job.slot0;
    b.n_slots = job.n_slots;
    b.jpb = 4 * JBW;
    b.n_blocks = b.n_slots * ((job.db.n_jb + b.jpb - 1) / b.jpb);
    b.first = total;
    total += round8(b.n_blocks);
  }
  a.n_jobs = (uint32_t)n;
  a.total = total;
  if (total == 0) return hipSuccess;
  hipExtLaunchKernelGGL(k_scan_b1r<JBW, D, NT>, dim3(total), dim3(256), 0, s, e0, e1, 0, a);
  return hipGetLastError();
}

// Blocks of a persistent batched launch: each takes about kItemsPerBlock work
// items, and a launch has at least kMinBlocks per wave-slot of occupancy
// (four per CU on 256 CUs) when it has that many items.
constexpr uint32_t kItemsPerBlock = 16, kMinBlocks = 1024;

template <int JBW, int CBW, int D, int OCC, int NW>
hipError_t run_mfma(const ScanJob *jobs, size_t n, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  constexpr uint32_t kAtomsChunk = kKCB * CBW;
  constexpr bool kDma = 3 * kAtomsChunk * 64 * 16 * OCC <= 160 * 1024;  // as in the kernel
  MfArgs a{};
  uint32_t total = 0;
  for (size_t i = 0; i < n; ++i) {
    const ScanJob &job = jobs[i];
    // the padded contraction steps past n_ib read database atoms beyond the
    // last row block of the last slot: they must stay inside the tail padding
    const uint32_t S = (std::max(job.db.n_ib, (kDma ? 3u : 2u) * kKCB) + D - 1) / D * D;
    if ((S - job.db.n_ib) * kAtomBytes > kDbTailBytes) return hipErrorInvalidValue;
    MfJob &m = a.jobs[i];
    m.db = job.db;
    m.qatoms = job.qatoms;
    m.out = job.out;
    m.B = job.B;
    m.n_cb = (2 * job.B + kCB - 1) / kCB;
    m.cb_stride = job.cb_stride ? job.cb_stride : m.n_cb;
    m.q_ibs = job.cb_major ? 1 : m.cb_stride;
    m.q_cbs = job.cb_major ? job.db.n_ib : 1;
    m.p_stride = job.p_stride ? job.p_stride : 2 * job.B * job.db.C;
    m.n_jg = (job.db.n_jb + NW * JBW - 1) / (NW * JBW);
    m.n_cbt = (m.n_cb + CBW - 1) / CBW;
    m.slot0 = job.slot0;
    m.n_items = job.n_slots * m.n_jg * m.n_cbt;
    // persistent blocks: about kItemsPerBlock items each, but never fewer
    // blocks than the chip holds at once
    m.n_blocks = std::max(std::min(m.n_items, kMinBlocks * OCC),
                          (m.n_items + kItemsPerBlock - 1) / kItemsPerBlock);
    m.first = total;
    total += round8(m.n_blocks);
  }
  a.n_jobs = (uint32_t)n;
  a.total = total;
  if (total == 0) return hipSuccess;
  bool one_tile = true;
  for (size_t i = 0; i < n; ++i) one_tile = one_tile && a.jobs[i].n_cbt == 1;
  if (one_tile)
    hipExtLaunchKernelGGL(k_scan_mfma<JBW, CBW, D, OCC, NW, true>, dim3(total),
                          dim3(64 * NW), 0, s, e0, e1, 0, a);
  else
    hipExtLaunchKernelGGL(k_scan_mfma<JBW, CBW, D, OCC, NW, false>, dim3(total),
                          dim3(64 * NW), 0, s, e0, e1, 0, a);
  return hipGetLastError();
}

typedef hipError_t (*ScanFn)(const ScanJob *, size_t, hipStream_t, hipEvent_t, hipEvent_t);

struct Variant {
  ScanCfg cfg;
  ScanFn fn;
};

// ScanCfg for kind 0: jbw, unr = k-blocks in flight, nt = nontemporal | ring << 1.
// ScanCfg for kind 1: jbw, unr = ring depth D, nt = log2(CBW) | (OCC - 1) << 4
// | (NW == 8) << 5.
#define MFW(J, C, D, O, W)                                                                 \
  {{1, J, D, (C == 8 ? 3 : C == 4 ? 2 : C == 2 ? 1 : 0) | ((O - 1) << 4) | ((W == 8) << 5)}, \
   run_mfma<J, C, D, O, W>}
#define MF(J, C, D, O) MFW(J, C, D, O, 4)
const Variant kVariants[] = {
    // batch-1 streaming, grouped loads and ring
    {{0, 8, 4, 1}, run_b1<8, 4, true>},  {{0, 4, 8, 1}, run_b1<4, 8, true>},
    {{0, 2, 8, 1}, run_b1<2, 8, true>},  {{0, 4, 4, 3}, run_b1r<4, 4, true>},
    {{0, 2, 8, 3}, run_b1r<2, 8, true>}, {{0, 4, 8, 3}, run_b1r<4, 8, true>},
    {{0, 2, 4, 3}, run_b1r<2, 4, true>}, {{0, 4, 2, 3}, run_b1r<4, 2, true>},
    // batched MFMA
    MF(1, 1, 8, 1), MF(2, 1, 8, 1), MF(4, 1, 8, 1), MF(4, 1, 8, 2),
    MF(1, 2, 8, 1), MF(2, 2, 8, 1), MF(4, 2, 8, 1), MF(2, 2, 8, 2),
    MF(1, 4, 8, 1), MF(2, 4, 8, 1), MF(2, 4, 4, 2), MF(2, 4, 8, 2), MF(4, 4, 8, 1), MF(4, 4, 4, 1),
    MF(1, 8, 8, 1), MF(2, 8, 8, 1), MF(2, 8, 4, 1), MF(1, 8, 4, 2), MF(1, 8, 8, 2),
    // eight waves per block, two per SIMD, sharing one query chunk (sixteen
    // waves of (1,4) tiles measured 3-5 % slower than eight of (2,4))
    MFW(1, 8, 8, 1, 8), MFW(1, 8, 4, 1, 8), MFW(2, 4, 8, 1, 8), MFW(2, 4, 4, 1, 8),
};
#undef MF
#undef MFW

// Column blocks per wave worth trying for a batch of B queries.
uint32_t cbw_for(uint32_t B) {
  const uint32_t n_cb = (2 * B + kCB - 1) / kCB;
  return n_cb >= 8 ? 8 : n_cb >= 4 ? 4 : n_cb >= 2 ? 2 : 1;
}

}  // namespace

std::vector<ScanCfg> scan_candidates(uint32_t B) {
  std::vector<ScanCfg> out;
  const uint32_t cbw = cbw_for(B);
  for (const Variant &v : kVariants) {
    const uint32_t vc = 1u << (v.cfg.nt & 15);
    if (B == 1 ? v.cfg.kind == 0 : (v.cfg.kind == 1 && (vc == cbw || 2 * vc == cbw)))
      out.push_back(v.cfg);
  }
  return out;
}

// From eight column blocks up, the eight-wave (2,4) tile with an 8-deep ring
// (fastest at B = 32 and 128); below, the four-wave (2, cbw) tile.
ScanCfg scan_default_mfma(uint32_t B) {
  const uint32_t cbw = cbw_for(B);
  if (cbw == 8) return ScanCfg{1, 2, 8, 2 | (1 << 5)};
  const uint8_t lg = cbw == 4 ? 2 : cbw == 2 ? 1 : 0;
  return ScanCfg{1, 2, 8, lg};
}

ScanCfg scan_default(uint32_t B) {
  if (B == 1) return ScanCfg{0, 4, 4, 3};
  return scan_default_mfma(B);
}

const char *scan_kernel_name(const ScanCfg &cfg, const DbDesc &d) {
  if (cfg.kind == 1) return "k_scan_mfma";
  const uint32_t tail = d.n_ib % kB1Chunk;
  const bool ring = (cfg.nt & 2) && (kB1Chunk / 2) % cfg.unr == 0 && (tail / 2) % cfg.unr == 0;
  return ring ? "k_scan_b1r" : "k_scan_b1";
}

hipError_t launch_scan(const ScanJob *jobs, size_t n, const ScanCfg &cfg, hipStream_t s,
                       hipEvent_t e0, hipEvent_t e1) {
  for (size_t i = 0; i < n; ++i) {
    const ScanJob &j = jobs[i];
    // the batch-1 kernel reads the NTT-form query; the batched kernel (any B) atoms
    if (cfg.kind == 0 ? (j.B != 1 || !j.q_ntt) : !j.qatoms) return hipErrorInvalidValue;
    if (j.n_slots == 0 || j.slot0 + j.n_slots > j.db.K * j.db.N) return hipErrorInvalidValue;
    if (j.cb_stride && j.cb_stride * kCB < 2 * j.B) return hipErrorInvalidValue;
    if (cfg.kind == 1 && j.p_stride && j.p_stride < 2 * j.B * j.db.C) return hipErrorInvalidValue;
  }
  for (const Variant &v : kVariants) {
    if (v.cfg.kind != cfg.kind || v.cfg.jbw != cfg.jbw || v.cfg.unr != cfg.unr || v.cfg.nt != cfg.nt)
      continue;
    for (size_t i = 0; i < n; i += kMaxFused) {
      const hipError_t e = v.fn(jobs + i, std::min<size_t>(kMaxFused, n - i), s, i == 0 ? e0 : nullptr,
                                i + kMaxFused >= n ? e1 : nullptr);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  return hipErrorInvalidValue;
}

}  // namespace pir
