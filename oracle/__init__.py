"""CPU oracle of the Jet refinement pass -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct implementations used to check the device
library: ``oracle.oracle`` (C, via ctypes) and ``oracle.micro`` (pure
Python, tiny graphs only). Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package. It shares no code
with the device library; both consume the seeded generators of
``paper_2304_13194_amd.inputs``.
"""
