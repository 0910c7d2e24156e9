"""Client side of the scan, for tests: one-hot RLWE queries and the end-to-end check.

A query for row ``i*`` is ``R`` ciphertexts, the ``i``-th encrypting the
constant polynomial ``[i == i*]`` -- the encrypted one-hot vector of
Sec. 2.5, with RLWE ciphertexts in place of LWE ones as in poly-HE folding
(Sec. 3.2).  Folding it against the database returns, for each column ``j``,
a ciphertext whose phase is ``Delta*DB[i*][j] + sum_i DB[i][j]*e_i``
(Eq. he-linear and the phase linearity of App. A), so decryption yields row
``i*`` while that sum stays below ``Delta/2``.
"""

from __future__ import annotations

import numpy as np

import synth

from . import rlwe


def onehot_query(seed: int, b: int, i_star: int, R: int, primes: list[int],
                 psis: list[int], delta: int, N: int) -> tuple[np.ndarray, np.ndarray]:
    """Encrypt the one-hot vector for row ``i_star``: returns ``(ct [R][2][K][N] uint64, s [N])``."""
    s = synth.secret(seed, b, N)
    m = np.zeros((R, N), dtype=np.int64)
    m[i_star, 0] = 1
    a = np.stack([synth.mask_row(seed, b, i, primes, N) for i in range(R)])   # [R][K][N]
    e = np.stack([synth.error_row(seed, b, i, N) for i in range(R)])          # [R][N]
    ct = rlwe.encrypt(m, s, a, e, primes, psis, delta)
    return ct, s


def decrypt_answers(ans_coeff: np.ndarray, s: np.ndarray, primes: list[int], psis: list[int],
                    delta: int, p: int) -> tuple[np.ndarray, np.ndarray]:
    """Decrypt ``[C][2][K][N]`` answer ciphertexts: ``(m [C][N], noise [C][N])``."""
    return rlwe.decrypt(ans_coeff, s, primes, psis, delta, p)
