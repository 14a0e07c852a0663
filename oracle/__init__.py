"""CPU oracle for the thin-film Ising Metropolis path (arXiv:1411.5588).

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the product package never does.
"""
