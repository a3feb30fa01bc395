"""CPU oracle of the SUPA propagation model (test infrastructure only).

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg import this package.  The product path (the HIP library and its Python
binding) never does, and this package imports nothing from the product.
"""
