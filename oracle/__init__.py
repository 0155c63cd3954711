"""CPU oracle for the epsilon self-join (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package. The product path (paper_1803_04120_amd) never does.
"""
