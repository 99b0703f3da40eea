"""Oracle -- test infrastructure only.

A plain, slow, FP64 CPU implementation of what the GPU path computes, written
from the paper: the particle-particle ladder (Sec. II.C) in plain C, and the
closed-shell RI-CCSD around it (Sec. II.A) plus the learned-guess network in
numpy.  Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg may import it.  It shares no code with the GPU path.
"""
