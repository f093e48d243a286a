"""Plain FP64 CPU oracle for Hermitian-symmetric CTMRG.

TEST INFRASTRUCTURE ONLY. Nothing in the library path imports, links or runs
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP implementation.

Contents
--------
basis       the bra-ket swap S, its eigenbasis U and the double layer
            (Sec. II A, II B of the paper).
ctmrg       directional CTMRG, in the plain (unrotated, one-sector) form and
            in the rotated Z2 form with per-sector truncated SVDs, plus the
            observables: one-site environment, RDMs, energy, Hermitian
            symmetry error, partition function per site (Sec. II A, II B, III A).
c4v         the C4v-symmetric CTMRG (one corner, one edge; Sec. II A).
hotrg       HOTRG in the plain and Z2 forms, with the symmetry probe b
            (Sec. II A, III A); its readings are listed in its docstring.
bruteforce  exact contraction of small finite open networks by row transfer,
            used to pin the CTMRG recursion where it is exact.

Readings of the paper where it is silent (the directional variant, the
initial environment, the projector formula, the truncation cutoff and the
normalisation) are listed in the docstrings of `ctmrg`.
"""
