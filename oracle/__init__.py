"""Plain, slow FP64 CPU oracle for the RPMD / adQTB hot path of Ple et al.,
"Routine Molecular Dynamics Simulations Including Nuclear Quantum Effects" (2022).

TEST INFRASTRUCTURE ONLY. This package exists to check the HIP implementation. Only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does. It shares no code with the HIP library: the two are written
separately from the paper, and only the seeded input generator (``synth``) feeds both.

Every function cites the passage it follows. Where the paper is silent, the reading
used is stated in the docstring. Parity status: every function is pinned by a
closed form, invariant, special case or brute force in ``tests/test_oracle_*.py``,
except the two constants noted "parity unpinned" in ``oracle/qtb.py`` (the adaptation
rate units and the absent finite-timestep corrections) and the water force constants.
"""
