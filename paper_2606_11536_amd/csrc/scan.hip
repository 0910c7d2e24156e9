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
//    components x 4 limbs (half the B columns) per B operand.  The block
//    splits the slot's query limbs straight from the NTT-form query into LDS;
//    each wave streams its database atoms from HBM with UNR k-blocks of loads
//    in flight before the first MFMA that needs them.
//  * k_scan_mfma (B > 1): v_mfma_i32_32x32x32_i8 over whole atoms.  A wave
//    owns JBW x 8 database rows and CBW x 8 query columns; database atoms come
//    through a register ring D contraction steps deep, query atoms through
//    double-buffered LDS chunks shared by the block's four waves.
#include <algorithm>

#include "device_util.h"
#include "pir_internal.h"

namespace pir {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr uint32_t kB1Chunk = 64;  // query ibs split into LDS per chunk (16 KiB)

// Scan launches take a table of up to kMaxFused jobs; the logical block
// index space is the concatenation of the jobs' spaces (job j owns logical
// blocks [first, first + blocks)).  A block finds its job by a uniform
// search of the table in the kernel-argument segment.
constexpr int kMaxFused = 8;

struct B1Job {
  DbDesc db;
  const uint32_t *q;  // NTT-form query [1][R][2][K][N]
  uint32_t *out;      // answer [1][C][2][K][N]
  uint32_t slot0, n_slots;  // slots scanned: [slot0, slot0 + n_slots)
  uint32_t jpb;       // jbs per block
  uint32_t first;     // first logical block of this job
};

struct B1Args {
  B1Job jobs[kMaxFused];
  uint32_t n_jobs, total;
};

template <typename Args>
__device__ __forceinline__ uint32_t find_job(const Args &a, uint32_t L) {
  uint32_t jid = 0;
#pragma unroll
  for (int j = 1; j < kMaxFused; ++j)
    if ((uint32_t)j < a.n_jobs && L >= a.jobs[j].first) jid = j;
  return jid;
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

template <int JBW, int UNR, bool NT>
__global__ __launch_bounds__(256) void k_scan_b1(const B1Args args) {
  __shared__ uint32_t sq[kB1Chunk * 64];
  const uint32_t Lg = xcd_logical(blockIdx.x, gridDim.x);
  if (Lg >= args.total) return;
  const B1Job &a = args.jobs[find_job(args, Lg)];
  const uint32_t L = Lg - a.first;
  const DbDesc &db = a.db;
  const uint32_t slot = a.slot0 + L % a.n_slots, jchunk = L / a.n_slots;
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
    // Split the slot's query residues into limb bytes: item (ibl, half, c, e4)
    // covers i = 32 (ib0+ibl) + 16 half + 4 e4 + u, u < 4, and writes one word
    // per limb b at LDS lane (half, 4c + b), bytes 4 e4 .. 4 e4 + 3.
    for (uint32_t idx = tid; idx < nib * 16; idx += 256) {
      const uint32_t ibl = idx >> 4, r = idx & 15;
      const uint32_t half = r >> 3, c = (r >> 2) & 1, e4 = r & 3;
      const uint32_t i0 = (ib0 + ibl) * 32 + half * 16 + e4 * 4;
      uint32_t v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        v[u] = (i0 + u < db.R) ? qbase[((size_t)(i0 + u) * 2 + c) * qrow] : 0u;
#pragma unroll
      for (uint32_t b = 0; b < 4; ++b) {
        uint32_t w = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) w |= ((v[u] >> (7 * b)) & 127u) << (8 * u);
        sq[((ibl * 2 + half) * 8 + c * 4 + b) * 4 + e4] = w;
      }
    }
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

  // Epilogue.  Lane holds rows 4*(lane>>4) + r (row = 4 jl' + a, a = r) of
  // column lane & 15 (= 4 cc + b).
  const uint32_t b = lane & 3, cc = (lane >> 2) & 3, jlp = lane >> 4;
  const uint32_t wb = P.w[b], wbsh = P.w_sh[b];
  const double inv_q = 1.0 / (double)q;
  const size_t KN = (size_t)db.K * db.N;
#pragma unroll
  for (int w = 0; w < JBW; ++w) {
    const uint32_t jb = jb_begin + wave + 4 * w;
    if (jb >= jb_end) break;
#pragma unroll
    for (int jh = 0; jh < 2; ++jh) {
      const v4i &A = acc[w][jh];
      const uint32_t u = limb_sum_mod(A[0], A[1], A[2], A[3], q, inv_q);
      const uint32_t s = quad_sum_mod(mul_shoup(u, wb, wbsh, q), q);
      const uint32_t j = jb * 8 + jh * 4 + jlp;
      if (b == 0 && cc < 2 && j < db.C) a.out[((size_t)j * 2 + cc) * KN + (size_t)k * db.N + t] = s;
    }
  }
}

// ---------------------------------------------------------------------------
constexpr uint32_t kKCB = 4;  // contraction atoms per staged query chunk

struct MfJob {
  DbDesc db;
  const uint8_t *qatoms;  // query atoms [K][N][n_ib][cb_stride]
  uint32_t *out;          // answer [B][C][2][K][N]
  uint32_t B, n_cb, cb_stride;
  uint32_t slot0, n_slots, n_jg, n_cbt;
  uint32_t ns, n_sg;      // slots per block, slot groups: logical blocks = n_sg * n_jg * n_cbt
  uint32_t first;
};

struct MfArgs {
  MfJob jobs[kMaxFused];
  uint32_t n_jobs, total;
};

// JBW database row blocks x CBW query column blocks per wave; the four waves of
// a block take consecutive row blocks of one slot.  The slot takes S steps
// (n_ib rounded up to the ring depth D; steps past n_ib meet zero query atoms
// and read valid padding memory); the database-atom ring requests step g + D
// while step g computes, and query atoms come through double-buffered LDS
// chunks of kKCB steps.  No load sits under a data-dependent branch, so the
// load counters stay exact.  (MfJob::ns > 1 is reserved for streaming several
// slots per block; the launcher sets 1.)
template <int JBW, int CBW, int D, int OCC>
__global__ __launch_bounds__(256, OCC) void k_scan_mfma(const MfArgs args) {
  static_assert(D % kKCB == 0, "ring depth must be a multiple of the query chunk");
  constexpr uint32_t kBuf = kKCB * CBW * 64;  // uint4 per LDS buffer
  constexpr uint32_t kPer = (kBuf + 255) / 256;
  __shared__ uint4 sq[2 * kBuf];
  const uint32_t Lg = xcd_logical(blockIdx.x, gridDim.x);
  if (Lg >= args.total) return;
  const MfJob &a = args.jobs[find_job(args, Lg)];
  const uint32_t L = Lg - a.first;
  const DbDesc &db = a.db;
  // column tiles of the same rows are adjacent, then row groups of one slot
  // group: a database atom's second read and a slot's query atoms hit L2
  const uint32_t cbt = L % a.n_cbt;
  const uint32_t rest = L / a.n_cbt;
  const uint32_t jg = rest % a.n_jg, sg = rest / a.n_jg;
  const uint32_t s_begin = a.slot0 + sg * a.ns;
  const uint32_t s_count = min(a.ns, a.slot0 + a.n_slots - s_begin);
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t n_ib = db.n_ib, n_jb = db.n_jb, n_cb = a.n_cb, cbs = a.cb_stride;
  const uint32_t cb0 = cbt * CBW;
  const uint32_t ncb = min((uint32_t)CBW, n_cb - cb0);
  const uint32_t S = (n_ib + D - 1) / D * D;  // steps per slot

  uint32_t jbs[JBW];
  bool jv[JBW];
  size_t row_off[JBW];
#pragma unroll
  for (int w = 0; w < JBW; ++w) {
    jbs[w] = (jg * 4 + wave) * JBW + w;
    jv[w] = jbs[w] < n_jb;
    // rows past C read row block 0: valid memory, results discarded
    row_off[w] = (size_t)(jv[w] ? jbs[w] : 0) * n_ib * kAtomBytes;
  }
  const size_t slot_stride = (size_t)n_jb * n_ib * kAtomBytes;
  const uint8_t *atoms_lane = db.atoms + lane * 16;
  // First atom of ring group (u, ks) for row block w; groups past the block
  // read the block's first atom (valid memory, never used).  Steps of a slot
  // past n_ib run into the following atoms or the allocation's tail padding
  // and meet zero query atoms.
  auto group_ptr = [&](int w, uint32_t u, uint32_t ks) {
    const bool ok = u < s_count;
    const size_t off = (size_t)(s_begin + (ok ? u : 0)) * slot_stride + row_off[w] +
                       (size_t)(ok ? ks : 0) * kAtomBytes;
    return atoms_lane + off;
  };
  const uint4 *qbase = reinterpret_cast<const uint4 *>(a.qatoms);
  // query atoms of the chunk starting at step ks of slot u (zero past the block)
  auto stage_load = [&](uint32_t u, uint32_t ks, uint4 (&st)[kPer]) {
    const bool uok = u < s_count;
    const uint4 *qs = qbase + (size_t)(s_begin + (uok ? u : 0)) * n_ib * cbs * 64;
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
      const uint32_t idx = tid + 256 * r;
      const uint32_t kk = idx / (CBW * 64), c = (idx / 64) % CBW, l = idx & 63;
      const bool ok = uok && idx < kBuf && ks + kk < n_ib && c < ncb;
      const uint4 v = qs[ok ? ((size_t)(ks + kk) * cbs + cb0 + c) * 64 + l : 0];
      st[r] = ok ? v : make_uint4(0, 0, 0, 0);
    }
  };
  auto stage_store = [&](uint4 *buf, const uint4 (&st)[kPer]) {
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r)
      if (tid + 256 * r < kBuf) buf[tid + 256 * r] = st[r];
  };
  v4i bcur[CBW], bnext[CBW];
  auto b_read = [&](const uint4 *src, v4i (&bv)[CBW]) {
#pragma unroll
    for (int c = 0; c < CBW; ++c) {
      const uint4 u = src[c * 64 + lane];
      bv[c] = v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
    }
  };

  v16i acc[JBW][CBW];
#pragma unroll
  for (int w = 0; w < JBW; ++w)
#pragma unroll
    for (int c = 0; c < CBW; ++c) acc[w][c] = v16i{};

  v4i ring[D][JBW];
#pragma unroll
  for (int w = 0; w < JBW; ++w) {
    const uint8_t *p = group_ptr(w, 0, 0);
#pragma unroll
    for (int d = 0; d < D; ++d)
      ring[d][w] = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(p + d * kAtomBytes));
  }
  uint4 st[kPer];
  stage_load(0, 0, st);
  stage_store(sq, st);
  __syncthreads();
  b_read(sq, bcur);

  // epilogue constants.  32x32 result: lane holds column lane & 31 (= 4 cc + b)
  // and, in register r, row 8*(r>>2) + 4*(lane>>5) + (r&3)  (row = 4 jl + a).
  const uint32_t b = lane & 3, cc = (lane >> 2) & 7, hi = lane >> 5;
  const size_t KN = (size_t)db.K * db.N;
  const uint32_t ncol = 2 * a.B;
  uint32_t chunk = 0;  // chunks completed (LDS buffer parity)

  {
    const uint32_t u = 0;
    for (uint32_t ks0 = 0; ks0 < S; ks0 += D) {
      // the group that refills the ring: next D steps of this slot or the next slot
      const bool same = ks0 + D < S;
      const uint32_t ur = same ? u : u + 1, kr = same ? ks0 + D : 0;
      const uint8_t *rp[JBW];
#pragma unroll
      for (int w = 0; w < JBW; ++w) rp[w] = group_ptr(w, ur, kr);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int kk = d % kKCB;
        if (kk == 0) {
          // next chunk, in flight during this one
          if (d + kKCB < D) stage_load(u, ks0 + d + kKCB, st);
          else stage_load(ur, kr, st);
        }
        if (kk + 1 < (int)kKCB) b_read(sq + (chunk & 1) * kBuf + (kk + 1) * CBW * 64, bnext);
#pragma unroll
        for (int c = 0; c < CBW; ++c)
#pragma unroll
          for (int w = 0; w < JBW; ++w)
            acc[w][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ring[d][w], bcur[c], acc[w][c], 0, 0, 0);
#pragma unroll
        for (int w = 0; w < JBW; ++w)
          ring[d][w] = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(rp[w] + d * kAtomBytes));
        if (kk == (int)kKCB - 1) {
          ++chunk;
          stage_store(sq + (chunk & 1) * kBuf, st);
          __syncthreads();
          b_read(sq + (chunk & 1) * kBuf, bnext);
        }
#pragma unroll
        for (int c = 0; c < CBW; ++c) bcur[c] = bnext[c];
      }
    }
  }
  {
    // the slot is complete: reduce and store
    const uint32_t slot = s_begin;
    const uint32_t k = slot >> db.log2n, t = slot & (db.N - 1);
    const DevPrime &P = db.primes[k];
    const uint32_t q = P.q;
    uint32_t wv[4], wsh[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      wv[r] = P.w[r + b];
      wsh[r] = P.w_sh[r + b];
    }
#pragma unroll
    for (int w = 0; w < JBW; ++w) {
#pragma unroll
      for (int c = 0; c < CBW; ++c) {
        const uint32_t col = (cb0 + c) * 8 + cc;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          // sum over limbs a in the lane (Shoup products), then over b across lanes
          uint32_t s2 = 0;
#pragma unroll
          for (int r = 0; r < 4; ++r)
            s2 += mul_shoup((uint32_t)acc[w][c][4 * qq + r], wv[r], wsh[r], q);
          s2 = csub(s2, 4 * q);
          s2 = csub(s2, 2 * q);
          const uint32_t sv = quad_sum_mod(s2, q);
          const uint32_t j = jbs[w] * 8 + 2 * qq + hi;
          if (jv[w] && (uint32_t)c < ncb && b == 0 && j < db.C && col < ncol)
            a.out[(((size_t)(col >> 1) * db.C + j) * 2 + (col & 1)) * KN + (size_t)k * db.N + t] = sv;
        }
      }
    }
  }
}

inline uint32_t round8(uint32_t x) { return (x + 7) / 8 * 8; }

template <int JBW, int UNR, bool NT>
hipError_t run_b1(const ScanJob *jobs, size_t n, hipStream_t s) {
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
    b.first = total;
    total += b.n_slots * ((job.db.n_jb + b.jpb - 1) / b.jpb);
  }
  a.n_jobs = (uint32_t)n;
  a.total = total;
  if (total == 0) return hipSuccess;
  k_scan_b1<JBW, UNR, NT><<<round8(total), 256, 0, s>>>(a);
  return hipGetLastError();
}

template <int JBW, int CBW, int D, int OCC>
hipError_t run_mfma(const ScanJob *jobs, size_t n, hipStream_t s) {
  MfArgs a{};
  uint32_t total = 0;
  for (size_t i = 0; i < n; ++i) {
    const ScanJob &job = jobs[i];
    MfJob &m = a.jobs[i];
    m.db = job.db;
    m.qatoms = job.qatoms;
    m.out = job.out;
    m.B = job.B;
    m.n_cb = (2 * job.B + kCB - 1) / kCB;
    m.cb_stride = job.cb_stride ? job.cb_stride : m.n_cb;
    m.slot0 = job.slot0;
    m.n_slots = job.n_slots;
    m.n_jg = (job.db.n_jb + 4 * JBW - 1) / (4 * JBW);
    m.n_cbt = (m.n_cb + CBW - 1) / CBW;
    // enough blocks to fill the chip several times over, each streaming up to
    // 16 slots so that only the first pays the pipeline fill
    const uint32_t per_slot = m.n_jg * m.n_cbt;
    (void)per_slot;
    const uint32_t ns = 1;  // one slot per block
    m.ns = ns;
    m.n_sg = (m.n_slots + ns - 1) / ns;
    m.first = total;
    total += m.n_cbt * m.n_sg * m.n_jg;
  }
  a.n_jobs = (uint32_t)n;
  a.total = total;
  if (total == 0) return hipSuccess;
  k_scan_mfma<JBW, CBW, D, OCC><<<round8(total), 256, 0, s>>>(a);
  return hipGetLastError();
}

typedef hipError_t (*ScanFn)(const ScanJob *, size_t, hipStream_t);

struct Variant {
  ScanCfg cfg;
  ScanFn fn;
};

// ScanCfg for kind 1: jbw, unr = ring depth D, nt = log2(CBW) | (OCC - 1) << 4.
#define MF(J, C, D, O) \
  {{1, J, D, (C == 8 ? 3 : C == 4 ? 2 : C == 2 ? 1 : 0) | ((O - 1) << 4)}, run_mfma<J, C, D, O>}
const Variant kVariants[] = {
    // batch-1 streaming: (kind 0, jbw, unroll, nontemporal)
    {{0, 8, 4, 0}, run_b1<8, 4, false>}, {{0, 8, 8, 0}, run_b1<8, 8, false>},
    {{0, 4, 4, 0}, run_b1<4, 4, false>}, {{0, 4, 8, 0}, run_b1<4, 8, false>},
    {{0, 2, 8, 0}, run_b1<2, 8, false>}, {{0, 8, 4, 1}, run_b1<8, 4, true>},
    {{0, 4, 8, 1}, run_b1<4, 8, true>},  {{0, 2, 8, 1}, run_b1<2, 8, true>},
    // batched MFMA
    MF(1, 1, 8, 1), MF(2, 1, 8, 1), MF(4, 1, 8, 1), MF(4, 1, 8, 2),
    MF(1, 2, 8, 1), MF(2, 2, 8, 1), MF(4, 2, 8, 1), MF(2, 2, 8, 2),
    MF(1, 4, 8, 1), MF(2, 4, 8, 1), MF(2, 4, 4, 2), MF(4, 4, 8, 1), MF(4, 4, 4, 1),
    MF(1, 8, 8, 1), MF(2, 8, 8, 1), MF(2, 8, 4, 1), MF(1, 8, 4, 2),
};
#undef MF

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

ScanCfg scan_default_mfma(uint32_t B) {
  const uint32_t cbw = cbw_for(B);
  const uint8_t lg = cbw == 8 ? 3 : cbw == 4 ? 2 : cbw == 2 ? 1 : 0;
  return ScanCfg{1, 2, 8, lg};
}

ScanCfg scan_default(uint32_t B) {
  if (B == 1) return ScanCfg{0, 2, 8, 1};
  const uint32_t cbw = cbw_for(B);
  const uint8_t lg = cbw == 8 ? 3 : cbw == 4 ? 2 : cbw == 2 ? 1 : 0;
  return ScanCfg{1, 2, 8, lg};
}

hipError_t launch_scan(const ScanJob *jobs, size_t n, const ScanCfg &cfg, hipStream_t s) {
  for (size_t i = 0; i < n; ++i) {
    const ScanJob &j = jobs[i];
    // the batch-1 kernel reads the NTT-form query; the batched kernel (any B) atoms
    if (cfg.kind == 0 ? (j.B != 1 || !j.q_ntt) : !j.qatoms) return hipErrorInvalidValue;
    if (j.n_slots == 0 || j.slot0 + j.n_slots > j.db.K * j.db.N) return hipErrorInvalidValue;
    if (j.cb_stride && j.cb_stride * kCB < 2 * j.B) return hipErrorInvalidValue;
  }
  for (const Variant &v : kVariants) {
    if (v.cfg.kind != cfg.kind || v.cfg.jbw != cfg.jbw || v.cfg.unr != cfg.unr || v.cfg.nt != cfg.nt)
      continue;
    for (size_t i = 0; i < n; i += kMaxFused) {
      const hipError_t e = v.fn(jobs + i, std::min<size_t>(kMaxFused, n - i), s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  return hipErrorInvalidValue;
}

}  // namespace pir
