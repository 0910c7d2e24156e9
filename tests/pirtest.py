"""Shared helpers for the GPU parity tests: workloads built from the seeded
generators, expected values from the oracle, transfers to and from the device."""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import synth
from oracle import params as op
from oracle import query as oq
from oracle import scan as osc


@dataclass
class Ring:
    log2n: int
    primes: list[int]
    psis: list[int]
    delta: int
    p: int = 256

    @property
    def N(self) -> int:
        return 1 << self.log2n

    @property
    def K(self) -> int:
        return len(self.primes)

    def pir_params(self):
        from paper_2606_11536_amd import pir
        return pir.Params(self.log2n, list(self.primes), 8)


def ring(log2n: int, K: int) -> Ring:
    N = 1 << log2n
    qs = op.ntt_primes(N, K)
    return Ring(log2n, qs, [op.psi_min(N, q) for q in qs], op.scale(qs, 256))


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to("cuda")


def to_host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32).astype(np.uint64)


def empty_dev(shape):
    import torch
    return torch.empty(shape, dtype=torch.int32, device="cuda")


def residues(rng: np.random.Generator, lead: tuple, rg: Ring) -> np.ndarray:
    """Uniform residues with layout [..., K, N]."""
    return np.stack([rng.integers(0, q, size=lead + (rg.N,), dtype=np.uint64) for q in rg.primes],
                    axis=-2)


def onehot_queries(seed: int, idx: np.ndarray, R: int, rg: Ring):
    """Encrypted one-hot queries: ([B][R][2][K][N] uint64, secrets [B][N])."""
    cts, secrets = [], []
    for b, i_star in enumerate(idx):
        ct, s = oq.onehot_query(seed, b, int(i_star), R, rg.primes, rg.psis, rg.delta, rg.N)
        cts.append(ct)
        secrets.append(s)
    return np.stack(cts), np.stack(secrets)


def sample_columns(C: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    extra = rng.choice(C, size=min(C, count), replace=False)
    return np.unique(np.concatenate([[0, C - 1], extra]))


def expected_columns(raw: np.ndarray, q_hat: np.ndarray, cols: np.ndarray, rg: Ring) -> np.ndarray:
    """Oracle NTT-form answer for the listed columns: [B][len(cols)][2][K][N]."""
    d_hat = osc.db_ntt(raw[:, cols, :], rg.primes, rg.psis)
    return osc.db_mul(d_hat, q_hat, rg.primes)


def freivalds_ok(raw: np.ndarray, q_hat: np.ndarray, ans: np.ndarray, rg: Ring, seed: int,
                 coeff_form: bool) -> bool:
    """Two Freivalds draws per prime over the whole answer [B][C][2][K][N]."""
    C = raw.shape[1]
    for k, (q, psi) in enumerate(zip(rg.primes, rg.psis)):
        for draw in range(2):
            r = synth.freivalds_vector(seed, draw, C, q)
            exp = osc.freivalds_expected(raw, q_hat, r, k, q, psi)          # NTT form
            if coeff_form:
                from oracle import ntt as on
                exp = on.intt(exp, q, psi)
            if not np.array_equal(osc.freivalds_observed(ans, r, k, q), exp):
                return False
    return True
