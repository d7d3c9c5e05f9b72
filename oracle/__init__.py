"""CPU oracle for the NTT family and the Groth16 quotient chain.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs anything in this package; only the tests, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code, header, table or
constant with the HIP library: it derives every constant (roots of unity,
coset powers, inverses, Montgomery factors) itself from the modulus and the
generator.

Two implementations of the same definitions:

* ``oracle.ref`` — Python integers, the definitional oracle for small n.
* ``oracle.coracle`` — ctypes wrapper of ``ntt_oracle.c``: plain C with
  4x64-bit limbs, Barrett reduction and POSIX threads, for large n and for
  timing.

Every function cites the passage of the paper it follows.  Parity pins (the
checks that tie the oracle to mathematics rather than to itself) live in
``tests/test_oracle_pins.py``.
"""
