"""Independent CPU oracle for the ray-shooting library: TEST INFRASTRUCTURE.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It never imports the GPU package and the GPU package never
imports it.
"""
