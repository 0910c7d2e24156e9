// Internal declarations of query expansion and RGSW folding (expand.hip,
// expand_api.cpp): gadget digits, the digit-key products and the combine steps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pir_internal.h"

namespace pir {

// The gadget and the CRT of a ciphertext modulus of one or two primes.
struct GadgetArgs {
  uint32_t K;                // 1 or 2
  uint32_t q0, q1;           // primes (q1 = 1 for K = 1)
  uint64_t Q;                // q0 q1
  double c;                  // q0^-1 mod q1 (K = 2)
  double inv_q0, inv_q1;     // 1 / q0, 1 / q1 (1 / q1 unused for K = 1)
  uint32_t base_log, n_digits;
};

// The signed permutation a polynomial goes through before its digits are
// taken: first the monomial product X^-shift, then the automorphism
// X -> X^g (g_inv = g^-1 mod 2N; g = 1 for none).
struct PolyMap {
  uint32_t shift, g_inv;
};

// Digits of polynomials, balanced base-2^base_log digits of the centred CRT
// value stored as residues mod q_k.
//  * expansion (diff = false): polynomial p = client * p_out + m takes input
//    k = m mod 2^level_bit of that client (src [clients][p_in][2][K][N],
//    coefficient form) on branch br = m >> level_bit (map m1 if br, else m0)
//    and writes the digits of component 0 of the mapped polynomial to
//    dig[p][n_digits][K][N];
//  * fold (diff = true): dig[p][2 n_digits][K][N] holds the digits of
//    components 0 and 1 of src[2p + 1] - src[2p].
hipError_t launch_gadget_digits(const uint32_t *src, uint32_t *dig, uint32_t n_polys,
                                uint32_t p_out, uint32_t p_in, uint32_t level_bit, PolyMap m0,
                                PolyMap m1, bool diff, uint32_t log2n, const GadgetArgs &g,
                                hipStream_t s);

// acc[p][c][k][t] = sum_d dig[p][d][k][t] key_p[d][c][k][t] mod q_k (NTT form),
// key_p = keys + (p / polys_per_key) * key_stride words; rows = digits per poly.
hipError_t launch_gadget_mac(const uint32_t *dig, const uint32_t *keys, size_t key_stride,
                             uint32_t polys_per_key, uint32_t *acc, uint32_t n_polys,
                             uint32_t rows, uint32_t log2n, uint32_t K, const DevPrime *primes,
                             hipStream_t s);

// Expansion: for output p = client * out_per_client + m (input k = m mod
// 2^level_bit, branch br = m >> level_bit, map m1 if br else m0), with c the
// input times X^-shift and tau(c_1) its component 1 through the automorphism:
//   out[p] = (c_0 + ks[p]_0, c_1 + tau(c_1) + ks[p]_1)
// src [B][P_in][2][K][N], ks and out [B][out_per_client][2][K][N], all in
// coefficient form.
struct CombineArgs {
  uint32_t B, P_in, level_bit, out_per_client;
};
hipError_t launch_expand_combine(const uint32_t *src, const uint32_t *ks, uint32_t *out,
                                 const CombineArgs &a, PolyMap m0, PolyMap m1, uint32_t log2n,
                                 uint32_t K, const uint32_t *q, hipStream_t s);

// Fold: out[p] = src[2p] + ext[p] (coefficient form, [..][2][K][N] each).
hipError_t launch_fold_combine(const uint32_t *src, const uint32_t *ext, uint32_t *out,
                               uint32_t n_polys, uint32_t log2n, uint32_t K, const uint32_t *q,
                               hipStream_t s);

// x <- x * f_k mod q_k for rows [n_rows][N] with row r of prime r % K.
hipError_t launch_scale_rows(uint32_t *x, size_t n_rows, uint32_t log2n, uint32_t K,
                             const uint32_t *q, const uint32_t *f, hipStream_t s);

}  // namespace pir
