"""CPU oracle for the projective-dynamics cloth step (TEST INFRASTRUCTURE).

A plain FP64 implementation written from the paper (arXiv 2403.19272:
Eq. (z), (local), (global), (exp), (query), (subspace_collision), (uu) and
Algorithm 1), used only by the tests, the smoke check and the CPU baseline of
the benchmark.  It shares no code with the HIP library: the two meet only in
the seeded scene generator, which holds none of the method's arithmetic.

Pins: every function here is checked by `-m "not gpu"` tests against closed
forms, library special cases, brute force and invariants (see tests/).
Parity unpinned: fidelity to the paper's own (unprinted) strain, bending and
collision-target models and constants; the paper prints no per-step values.
"""
