"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference implementations that the GPU library
is checked against.  Nothing here is imported by the product package; only
tests/, the smoke check and the bench's CPU-baseline leg use it.  It shares no
code with the GPU path: the only common inputs are the seeded scene arrays of
`mrs_inputs`.
"""
