"""CPU oracle for non-RNS CKKS/BGV homomorphic multiplication (test infrastructure).

A plain, slow, exact reference written from the paper's definitions, using only
Python's arbitrary-precision integers, the standard ``decimal`` module (as an exact
big-number multiplier) and numpy (for the floating-point CKKS encoding helper and
the fast textbook NTT).  It uses no number-theoretic transform or residue number
system on the exact scheme path.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it, and it shares no code,
table or constant with the GPU library.

Modules
-------
limbs   limb codec: integers <-> little-endian uint32 limb arrays (radix 2^32 form).
ring    negacyclic product in Z[X]/(X^N+1), literal schoolbook and Kronecker form.
ntt     negacyclic NTT / iNTT by definition and by textbook radix-2 recursion.
crt     CRT composition and Garner's mixed-radix conversion.
scheme  CKKS/BGV: keygen, encode/decode, encrypt/decrypt, tensor, relinearize, rescale.
"""
