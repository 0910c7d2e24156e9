// Internal declarations of libpir: device-side constants, the tile layouts
// of the scan, and the launchers the host API calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/pir.h"

namespace pir {

// ---------------------------------------------------------------------------
// Per-prime constants kept in device memory (one entry per RNS prime).
//   tw: [4][N] uint32 -- psi^brv(i), its Shoup companion, psi^-brv(i), its
//   Shoup companion, for i in [0, N); brv over log2 N bits.
//   w:  limb weights 2^(7s) mod q for s = 0..6 (index 7 unused), w_sh their
//   Shoup companions floor(w * 2^32 / q).
// ---------------------------------------------------------------------------
struct DevPrime {
  uint32_t q;
  uint32_t ninv, ninv_sh;
  uint32_t log2n;
  uint32_t w[8];
  uint32_t w_sh[8];
  const uint32_t *tw;
};

// ---------------------------------------------------------------------------
// Scan layouts.  Both operands of the scan are stored as 1 KiB "atoms", each
// holding exactly the bytes one 64-lane wave feeds to one
// v_mfma_i32_32x32x32_i8 operand: lane l owns bytes [16 l, 16 l + 16).
//
// An element x < 2^28 is split into four 7-bit limbs x = sum_a x_a 2^(7a),
// x_a in [0, 127], each a non-negative int8.
//
// Database atom (k, t, jb, ib): lane l = 32 g + 4 jl + a (g < 2, jl < 8,
// a < 4) holds limb a of D_t[j = 8 jb + jl][i = 32 ib + 16 g + e], e < 16,
// where D_t[j][i] is slot t (prime k) of NTT(lift(DB[i][j])).  Atom order
// [k][t][jb][ib]; jb < C_pad/8, ib < R_pad/32 (R_pad a multiple of 64).
//
// Query atom (k, t, ib, cb): lane l = 32 g + 4 cc + b holds limb b of
// Q_t[i = 32 ib + 16 g + e][col = 8 cb + cc], col = 2 * query + component.
// Atom order [k][t][ib][cb]; cb < ceil(2B/8).
//
// Because lane l feeds the same 16 k-indices of the contraction to the A and
// B operands, the MFMA's internal order of k is irrelevant: every row of A is
// matched with the same i-range of B.
// ---------------------------------------------------------------------------
constexpr uint32_t kAtomBytes = 1024;
constexpr uint32_t kJB = 8;    // database rows j per atom
constexpr uint32_t kIB = 32;   // contraction indices i per atom
constexpr uint32_t kRAlign = 64;
constexpr uint32_t kCB = 8;    // query columns per atom

// Bytes of padding after a database's last atom: the batched scan's padded
// contraction steps may read (never use) atoms there.
constexpr uint32_t kDbTailBytes = 64u << 10;

inline uint32_t r_pad(uint32_t R) { return (R + kRAlign - 1) / kRAlign * kRAlign; }
inline uint32_t c_pad(uint32_t C) { return (C + kJB - 1) / kJB * kJB; }

// Device-side description of one loaded database for the scan kernels.
struct DbDesc {
  const uint8_t *atoms;    // database atoms
  const DevPrime *primes;  // [K]
  uint32_t R, C, N, K, log2n;
  uint32_t n_jb, n_ib;     // C_pad / 8, R_pad / 32
};

// ---------------------------------------------------------------------------
// Launchers (implemented in the .hip files).  All are asynchronous on `s`.
// ---------------------------------------------------------------------------
// In-place forward / inverse NTT of rows [n_rows][N], row r uses prime r % K.
// add (inverse only, may be null): the rows are answers [..][2][K][N] and
// rows of component 1 first get the matching row of add ([..][K][N]) added.
hipError_t launch_ntt(uint32_t *data, size_t n_rows, uint32_t K, uint32_t log2n,
                      const DevPrime *primes, bool inverse, hipStream_t s,
                      const uint32_t *add = nullptr);
// Out-of-place forward NTT: src and dst both [n_rows][N] (row r -> prime r % K).
// Fused inverse NTT and modulus switching of n_polys answer polynomials
// [K][N] (K = 1 or 2, host primes q[K]) into [N] words mod 2^bits each.
hipError_t launch_intt_switch(const uint32_t *src, uint32_t *dst, size_t n_polys, uint32_t K,
                              const uint32_t *q, uint32_t log2n, const DevPrime *primes,
                              uint32_t bits, hipStream_t s, const uint32_t *add = nullptr);
// G = NTT(Delta iota(b)) of ring packing: b [B][D1] uint32 cut into Cp chunks
// of N, out [B][Cp][K][N]; delta[k] = Delta mod q_k.
hipError_t launch_offset_ntt(const uint32_t *b, uint32_t *out, uint32_t B, uint32_t D1,
                             uint32_t Cp, uint32_t K, uint32_t log2n, const DevPrime *primes,
                             const uint32_t *delta, hipStream_t s);
// Lift + forward NTT of uint32 rows (the ring-packing hint), as launch_lift_ntt.
hipError_t launch_lift_ntt32(const uint32_t *raw, uint32_t *out, uint32_t S, uint32_t s_valid,
                             uint32_t C, uint32_t K, uint32_t log2n, const DevPrime *primes,
                             hipStream_t s);
// Transpose a [rows][cols] uint32 matrix into out [cols][out_rows] (out_rows
// >= rows; entries past `rows` are zero).
hipError_t launch_transpose32(const uint32_t *in, uint32_t *out, uint32_t rows, uint32_t cols,
                              uint32_t out_rows, hipStream_t s);
// Scalar-HE database GEMM mod 2^32 (sgemm.hip): database int8 [D1][D0] into
// atoms [n_rb][n_kb]; queries uint32 [B][D0] into digit atoms [n_kb][n_cb];
// out [B][D1] = DB Q^T mod 2^32.  n_kb a multiple of 8, n_cb of 4.
hipError_t launch_sdb_pack(const int8_t *db, uint8_t *atoms, uint32_t D1, uint32_t D0,
                           uint32_t n_rb, uint32_t n_kb, hipStream_t s);
hipError_t launch_sq_pack(const uint32_t *q, uint8_t *atoms, uint32_t B, uint32_t D0,
                          uint32_t n_kb, uint32_t n_cb, hipStream_t s);
hipError_t launch_sgemm(const uint8_t *db, const uint8_t *q, uint32_t *out, uint32_t D1,
                        uint32_t B, uint32_t n_rb, uint32_t n_kb, uint32_t n_cb, hipStream_t s,
                        hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_ntt_copy(const uint32_t *src, uint32_t *dst, size_t n_rows, uint32_t K,
                           uint32_t log2n, const DevPrime *primes, hipStream_t s);
// Lift + forward NTT of a slab of raw database rows: raw [S][C][N] uint8 ->
// out [K][S][C][N] uint32.  Rows >= s_valid are taken as zero.
hipError_t launch_lift_ntt(const uint8_t *raw, uint32_t *out, uint32_t S, uint32_t s_valid,
                           uint32_t C, uint32_t K, uint32_t log2n, const DevPrime *primes,
                           hipStream_t s);
// Pack a slab (rows [i0, i0 + S)) of NTT-form database [K][S][C][N] into atoms.
hipError_t launch_pack_db(const uint32_t *ntt_slab, uint8_t *atoms, uint32_t i0, uint32_t S,
                          uint32_t R, uint32_t C, uint32_t N, uint32_t K, hipStream_t s);
// Read back canonical NTT-form database polys [ni][nj][K][N].
hipError_t launch_read_db(const DbDesc &db, uint32_t i0, uint32_t ni, uint32_t j0, uint32_t nj,
                          uint32_t *out, hipStream_t s);
// Pack NTT-form queries [B][R][2][K][N] into query atoms (R_pad rows).
hipError_t launch_pack_query(const uint32_t *q_ntt, uint8_t *qatoms, uint32_t B, uint32_t R,
                             uint32_t N, uint32_t K, hipStream_t s);
// Pack one NTT-form query [R][2][K][N] into columns 2*col_slot, 2*col_slot+1
// of column-block-major query atoms [K][N][n_cb][n_ib] (ScanJob::cb_major),
// touching no other column's bytes.
hipError_t launch_pack_query_slot(const uint32_t *q_ntt, uint8_t *qatoms, uint32_t col_slot,
                                  uint32_t n_cb, uint32_t R, uint32_t N, uint32_t K,
                                  hipStream_t s);

// One scan job for the scan kernels: the slots [slot0, slot0 + n_slots) of
// the flat slot index k * N + t (all K*N slots for a whole scan).
struct ScanJob {
  DbDesc db;
  const uint8_t *qatoms;   // query atoms of this job (batched kernel)
  const uint32_t *q_ntt;   // NTT-form query [1][R][2][K][N] (batch-1 kernel)
  // Answers, NTT form.  Batch-1 kernel: [B][C][2][K][N].  Batched kernel:
  // slot-major, answer polynomial p = (b C + j) 2 + c of slot s at
  // out[s * p_stride + p] (s = k N + t), so that a block's stores are whole
  // contiguous runs; launch_unpack_answers restores [B][C][2][K][N].
  uint32_t *out;
  uint32_t B;
  uint32_t slot0, n_slots;
  uint32_t cb_stride;      // column blocks per (k, t, ib) in qatoms; 0 = ceil(2B/8)
  uint32_t p_stride;       // batched kernel: row pitch of out in words; 0 = 2 B C
  // batched kernel: qatoms ordered [K][N][cb_stride][n_ib] (1) instead of
  // [K][N][n_ib][cb_stride] (0), so that one column block's atoms are contiguous
  uint32_t cb_major;
};

// A scan kernel variant.  kind 0: batch-1 streaming kernel (jbw row blocks per
// wave, unr k-blocks of loads in flight, nt = non-temporal loads); kind 1:
// batched MFMA kernel (jbw row blocks per wave, unr = database-atom ring
// depth, nt = log2 of the query column blocks per wave in bits 0-3 and the
// minimum waves per SIMD less one in bits 4-7).
struct ScanCfg {
  uint8_t kind, jbw, unr, nt;
};

std::vector<ScanCfg> scan_candidates(uint32_t B);
ScanCfg scan_default(uint32_t B);
// Default batched-kernel (kind 1) variant for B columns pairs, including B = 1.
ScanCfg scan_default_mfma(uint32_t B);
// Name of the kernel that variant cfg launches for database d.
const char *scan_kernel_name(const ScanCfg &cfg, const DbDesc &d);
// Scan every job with one variant; jobs are fused into launches of up to 8.
// kind 0 needs B == 1 for every job, kind 1 any B (query atoms).
// e0 / e1 (optional) are recorded by the first launch's start and the last
// launch's end.
hipError_t launch_scan(const ScanJob *jobs, size_t n, const ScanCfg &cfg, hipStream_t s,
                       hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Pseudo-random words (bytes < 128, words < 2^28) for autotuner timing runs.
hipError_t launch_fill_tuning(uint32_t *p, size_t n_words, hipStream_t s);

// Polynomials p0 .. p0 + P - 1 of a slot-major answer block sm ([KN][p_stride])
// into polynomial-major out ([P][KN]); KN must be a multiple of 64.
hipError_t launch_unpack_answers(const uint32_t *sm, uint32_t p_stride, uint32_t p0, uint32_t P,
                                 uint32_t KN, uint32_t *out, hipStream_t s);

// The library's fixed device scratch array (pir_answer_batch_static): its
// size, and its address on `device`, which must be the current device.  The
// address is looked up once per device and kept.
constexpr size_t kStaticScratchBytes = PIR_STATIC_SCRATCH_BYTES;
hipError_t static_scratch_init(int device, void **ptr);

}  // namespace pir
