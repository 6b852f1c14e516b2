"""Reference oracle for the colour-ordered Berends-Giele recursion.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
CPU evaluation of what the GPU path computes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (``paper_2502_07060_amd``) never imports it and
shares no code with it; the only common module is the seeded input generator
``paper_2502_07060_amd.inputs``, which holds none of the recursion's
arithmetic.

Modules
-------
fields        exact F_p (Python ints), FP64 complex (Python complex) and Q
              (fractions.Fraction) arithmetic behind one small interface.
bg            the recursion itself (paper Sec. 2.2, the current recursion and
              the 3-/4-gluon vertices), memoised over contiguous sub-ranges;
              mostly-minus or alternating metric (paper Sec. 3.1).
feynman       brute-force sum over colour-ordered Feynman diagrams with full
              vertex tensors -- an independent pin for ``bg``.
states        the d-dimensional polarisation states of paper Sec. 2.3 and
              their duals (square-root-free normalisation).
rational      residues of rationals, Chinese remaindering and rational
              reconstruction (F_p samples back to Q).
ffops         standalone batched F_p contractions and division.

Parity status per function is stated in each module header.
"""
