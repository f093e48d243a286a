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
cell        directional CTMRG on an Lx x Ly unit cell of different tensors,
            both forms (its readings are listed in its docstring).
complex_z2  complex tensors in the real representation of their Hermitian
            structure: real even-total and imaginary odd-total blocks, the
            product with f = [1, i] (Sec. II C).
c4v         the C4v-symmetric CTMRG (one corner, one edge; Sec. II A).
hotrg       HOTRG in the plain and Z2 forms, with the symmetry probe b
            (Sec. II A, III A); its readings are listed in its docstring.
bruteforce  exact contraction of small finite open networks by row transfer,
            used to pin the CTMRG recursion where it is exact.

Each module is pinned against what the paper and the mathematics fix (the
paper's worked example, brute-force contraction, Onsager's and Yang's
closed forms, Eckart-Young, infinite cylinders solved by their transfer
matrices) in tests/test_oracle_*.py.

Readings of the paper where it is silent (the directional variant, the
initial environment, the projector formula, the truncation cutoff and the
normalisation) are listed in the docstrings of `ctmrg`.
"""
