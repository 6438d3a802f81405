"""CPU oracle for population annealing on the 2D Ising model.

TEST INFRASTRUCTURE ONLY: plain, slow reference code used by the test suite,
the smoke check and the CPU-baseline leg of the benchmark.  Nothing in the
library imports it.
"""
