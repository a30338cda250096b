"""CPU oracle for the symmetry-adapted HEOM hot path.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import, call or execute anything in this
package; the product path never does, and this package imports nothing from
the product.

Contents (plain, slow, obviously correct; complex128/float64 throughout):

* conventional  -- the conventional scaled HEOM over every molecule-resolved
                   label n with |n| <= L and dense (N+1)x(N+1) ADOs
                   (paper Eq. scaled-HEOM), plus cavity loss and the optional
                   terminator; tiny N only.
* patterns      -- canonical occupation patterns (Sec. IV), categories and
                   multiplicities (Eqs. Mq, M0), unique-variable layout
                   (Sec. V.A), closed-form counts.
* uvar          -- the unique-variable generator M_u (Eq. uvar-propagator),
                   assembled row by row from the commutator with H_S summed
                   over molecules grouped by category (Sec. V.C.2) and from the
                   aligned target accessor (Eqs. aligned-accessor, uvar-up,
                   uvar-down); expansion to / compression from the
                   conventional hierarchy (Eq. central-covariance).
* integrate     -- classical fourth-order Runge-Kutta.
* observables   -- populations from a dense rho_S (definitions) and from the
                   tier-0 unique variables (Sec. V.D).

Parity status of every function is recorded in its docstring; none is
"parity unpinned".
"""
