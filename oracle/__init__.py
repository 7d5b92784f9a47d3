"""CPU oracle of the spin-1/2 / spin-1 CF4 solver: test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.
"""
