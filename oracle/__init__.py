"""Plain CPU FP64 oracle for the CFF/Yn pseudospectral shell method (Bruegmann,
"A pseudospectral matrix method for time-dependent tensor fields on a
spherical shell", arXiv:1104.3408).

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test
suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import it.  It shares no code with the HIP library: every matrix, table and
step here is rebuilt from the paper's definitions, in numpy/scipy FP64, without
blocking, fusion or reordering beyond what the paper states.

Modules (each function cites the section/equation it follows):
  grid          collocation grid (Sec. 2.1), differentiation matrices (Sec. 2.3),
                time-step rule (Sec. 4.1, Tab. dtfac)
  derivs        3-d spectral derivatives with the theta double cover (Sec. 2.1,
                2.4) and the Cartesian chain rule (Sec. 2.2, eq. dvdx)
  swsh          spin-weighted associated Legendre functions from Wigner d
                (Sec. 3.3), pseudo-inverse filter matrices (Sec. 3.2, 3.5)
  tensor_filter Y, Yg and Yn filters on the tetrad decomposition (Sec. 3.4, 3.5)
  ghg           first-order generalized-harmonic right-hand side and the
                freezing-incoming outer boundary condition (App. A.1, A.2)
  initial_data  Kerr-Schild data with numerical Phi, Pi and static gauge (App. A.3)
  evolve        classical RK4 method of lines with the filter after each step
                (Sec. 2.5)
  nested        shells coupled at shared spheres by characteristic upwinding
                (reading of the outlook of Sec. 1 / Sec. 5 with App. A.2)
  rounding      the angular products in the rounding of the reduced-precision
                modes (FP32, BF16x3 split products, plain bfloat16)

Parity pins: every function is checked in ``tests/test_oracle_*.py`` against
values the paper prints, closed forms, invariants or brute force.  The only
function without such a pin is the 58-field gauge-source extension in ``ghg``
(the paper gives no evolution equation for H_a, see ``ghg.rhs``), which is
marked "parity unpinned" there.
"""
