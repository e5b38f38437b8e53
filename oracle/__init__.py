"""Plain FP64 CPU oracle for the ETD schemes of Luo, Qiao and Zhao,
"Exponential Time Differencing Schemes for a Phase-Field Model of
Multicomponent Membranes".

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
runs this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the GPU library (no kernels,
headers, tables or helpers); the two meet only through seeded input arrays.

Modules
  core     grid, own DFT (naive exact-index mode + library FFT mode),
           spectral symbols, finite-difference operators, phi-functions
  fixed    fixed-membrane localization-split ETD1/ETDRK2 (Section 2)
  coupled  coupled stabilized spectral ETD1/ETDRK2, Algorithm 1 (Section 3)
  band     narrow-band index lists and the recovery step

Every function is pinned by a CPU test against something other than
itself (brute force, closed forms, theorems of the paper, invariants,
first variations of the energies); the coupled module's header lists its
pins.
"""
