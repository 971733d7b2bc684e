"""CPU oracle for the pseudo-spectral Navier-Stokes + Cahn-Hilliard step.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP implementation in ``paper_2406_01322_amd``.
"""
