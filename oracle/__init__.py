"""CPU oracle for the RLWE-PIR first-dimension scan -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously-correct reference that the GPU
library is checked against.  It is written from the paper's definitions and
shares no code with the GPU library (no kernels, headers, tables, constant
generators or pre/post-processing); the only code both sides use is the
seeded input generator in ``synth``.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import it; the product path never
does.

Modules
-------
``params``  RNS primes, roots of unity, scale (App. A, RNS prime selection; App. A.2).
``ntt``     schoolbook negacyclic product, the NTT by its definition, and a
            plain radix-2 NTT pinned to it (Sec. 2.3).
``rlwe``    toy RLWE encryption and decryption with CRT (App. A.2).
``scan``    plaintext lift + NTT of the database (Sec. 2.4), the
            first-dimension scan by its definition (Sec. 3.2 poly-HE folding,
            Sec. 4 INT32 modular GEMM), and a Freivalds full-output check.
``modswitch`` modulus switching of answers from Q down to 2^t (Sec. 4.3,
            App. D.5) and decryption at the reduced modulus.
``scalar``  the scalar-HE database GEMM mod 2^32 (Sec. 4.1) and a toy
            SimplePIR round trip (Sec. 2).
``pack``    Tiptoe-style ring packing of LWE ciphertexts into RLWE ones,
            H C + (0|G) (App. C.1, Eq. tiptoe-rp; Sec. 3.5).
``expand``  automorphisms, gadget digits and key switching; the recursive
            query expansion of ExpPack (Sec. 3.5, App. C.2); RGSW external
            products, CMux and folding (Sec. 3.2 step 7, Sec. 3.6).

All arithmetic is on exact integers (Python ints, or numpy uint64/int64 with
every intermediate bounded below 2**63); nothing is approximated.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against something other than itself (closed forms, sympy, brute force on
tiny inputs, the convolution theorem, the decryption of the selected row).
"""
