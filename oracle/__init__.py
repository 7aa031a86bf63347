"""CPU oracle (FP64, NumPy/SciPy) for the first-order Stokes assembly path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares no
code with the HIP path; only the seeded input generators (fo_inputs) serve both.
"""
