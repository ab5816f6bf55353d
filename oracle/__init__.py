"""CPU oracle for the multivariate discrete Walsh transform on digital nets.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (no headers, tables, helpers or generated constants) and imports
nothing from it.

The subpackage ``oracle.fast`` is the exception to "slow": a C + OpenMP
float64 restatement of the fast algorithms (Algorithms 1 and 2 and the
spectral routes of Sections 3.2 and 4), pinned to the definitions here at
small sizes and used where every output of a full-size run is compared.  It
too shares no code with the HIP library.

Every other function is a plain, slow restatement of a definition or closed
form of Liu, Dick and Hickernell, "A Multivariate Fast Discrete Walsh Transform
with an Application to Function Interpolation" (Mathematics of Computation),
computed in float64 / complex128 / int64, and never uses the fast algorithms
(Algorithms 1 and 2): transforms are the direct O(N^2) sums of their definitions, spline
coefficients come from a dense solve of the interpolation system, and ANOVA
variances from the direct double sums.  Each function cites the passage it
follows by section and equation label.

Pins (tests/test_oracle_*.py) tie each function to something other than
itself: textbook special cases (van der Corput, Sylvester-Hadamard, the
digit-tensor DFT), brute-force enumeration, invariants stated in the paper,
closed forms, and the analytic values the paper prints in Tables 1 and 2.
"""
