"""FP64 CPU oracle of the ultra-relativistic lattice Boltzmann update and the
exact ideal-fluid Riemann solution.

TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package.
"""
