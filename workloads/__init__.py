"""Seeded input generators shared by the oracle and the HIP path.

This package produces *inputs only*: cut circuits (gate lists, cut positions
and the segment-to-subcircuit assignment a cut searcher would return) and
synthetic subcircuit entry tensors shaped like the post-processing workloads
of the paper's runtime study, which fed random numbers to the reconstructor
(Section 5.4).  It holds none of the reconstruction arithmetic: no
attribution, no Kronecker sum, no dynamic-definition logic.
"""
