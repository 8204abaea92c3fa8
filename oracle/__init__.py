"""CPU oracles for batch SHA-3 -- TEST INFRASTRUCTURE ONLY.

``keccak_ref`` is the bit-level definition (numpy, Python loops over lanes);
``o2`` binds the lane-level C oracle ``keccak_o2.c``.  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import this package.
Neither oracle shares code with the HIP library.
"""
