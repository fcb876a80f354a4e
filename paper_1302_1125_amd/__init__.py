"""MI355X (gfx950) implementation of the per-cell, per-timestep update of the
ultra-relativistic lattice Boltzmann model of Mohseni, Mendoza, Succi and
Herrmann (arXiv:1302.1125): a HIP library with a C ABI (include/rlb.h) and a
thin Python binding (paper_1302_1125_amd.rlb)."""

__all__ = ["rlb", "workloads"]
