"""CPU FP64 oracle of the H^2 strong recursive skeletonization factor/solve.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct numpy code written
from the paper; it shares no code with the GPU library.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import it.
"""
