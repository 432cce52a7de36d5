"""FP64 CPU oracle for the HISQ Dslash / CG path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the GPU
library: its Dslash is a plain C loop over lexicographic sites
(``hisq_oracle.c``), its dense check builds the operator matrix entry by entry
(``dense.py``), its solvers are textbook loops in NumPy (``hisq.py``) and its
learned-preconditioner reference is written with whole-lattice NumPy shifts
(``ptc.py``).
"""
