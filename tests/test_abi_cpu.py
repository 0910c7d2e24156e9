"""Host-only checks of the C ABI (no GPU needed).

* libpir.so loads and exports every function include/pir.h declares;
* the library's prime search and root of unity (its own algorithms) agree
  with the oracle's (trial division, ascending search);
* parameter validation returns the documented status codes;
* without a GPU, creating a context fails with PIR_ERR_DEVICE (no fallback).
"""

import ctypes as ct
import os
import re
import subprocess

import pytest

from oracle import params as oparams
from paper_2606_11536_amd import pir

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pir.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pir_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["pir_db_load_ntt", "pir_ntt", "pir_intt", "pir_db_mul", "pir_answer_batch"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", pir.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pir_[a-z0-9_]+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    assert set(pir.SIGNATURES) == set(declared_functions())


@pytest.mark.parametrize("log2n,count", [(10, 2), (11, 2), (12, 2), (4, 3)])
def test_find_primes_matches_oracle(log2n, count):
    assert pir.find_primes(log2n, count, 28) == oparams.ntt_primes(1 << log2n, count)


@pytest.mark.parametrize("log2n,K", [(10, 1), (10, 2), (11, 2), (12, 2)])
def test_psi_matches_oracle(log2n, K):
    qs = oparams.ntt_primes(1 << log2n, K)
    assert pir.params_check(pir.Params(log2n, qs)) == [oparams.psi_min(1 << log2n, q) for q in qs]


def _status(p):
    return pir.lib.pir_params_check(ct.byref(p.c()), None)


def test_params_validation_codes():
    q = oparams.ntt_primes(2048, 2)
    assert _status(pir.Params(11, q)) == 0
    assert _status(pir.Params(9, oparams.ntt_primes(512, 1))) == 2      # N too small
    assert _status(pir.Params(13, q)) == 2                               # N too large
    assert _status(pir.Params(11, [q[0] + 4096])) == 2                   # not prime
    assert _status(pir.Params(11, [(1 << 28) + 1])) == 2                 # too big
    assert _status(pir.Params(11, [q[0], q[0]])) == 1                    # repeated
    assert _status(pir.Params(11, q, plain_log2=32)) == 0
    assert _status(pir.Params(11, q, plain_log2=33)) == 2
    assert _status(pir.Params(11, q, plain_log2=0)) == 2
    assert pir.lib.pir_params_check(None, None) == 1
    assert pir.lib.pir_find_primes(11, 0, 28, None) == 1


def test_scan_kernel_rejects_null_arguments():
    assert pir.lib.pir_scan_kernel(None, None, 1) is None
    assert pir.lib.pir_profile_stages(None, 4) == 1


def test_status_strings():
    for code, name in pir.STATUS.items():
        assert pir.lib.pir_status_string(code).decode() == name


def test_no_gpu_means_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ct.c_void_p()
    assert pir.lib.pir_ctx_create(0, 0, ct.byref(h)) == 5
    with pytest.raises(pir.PirError):
        pir.Context(0)
