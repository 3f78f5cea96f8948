"""CPU oracle for the stratified Cox hot path -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's cpu_baseline leg may import
this package.  It is independent of the HIP path and never imports it.
"""
