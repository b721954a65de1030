"""CPU oracle of the microcircuit simulation: test infrastructure only.

Imported by the test suite, the smoke check and the benchmark's CPU-baseline
leg; never by the simulator library or its Python binding.
"""
