"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This package only *draws* inputs: one- and two-electron integrals with the
statistics of the paper's workloads (PAH pi-systems and iron-sulfur clusters,
Sec. "Preparation of benchmark systems") and random spin-adapted matrix product
states of a prescribed bond dimension.  It contains none of the method's
arithmetic (no Hamiltonian application, no environments, no contraction); the
only linear algebra here is a QR factorisation that turns random Gaussian
blocks into isometries, and the counting that decides which symmetry sectors a
bond may carry.
"""
