"""CPU oracle for the xTC three-body folding (test infrastructure only).

Plain, slow, FP64 numpy implementations of what the GPU path computes,
written from the paper (Christlmaier et al., "xTC: An efficient treatment of
three-body interactions in transcorrelated methods"):

* ``jastrow``      -- u(r12), u'(r12) and the gradient of u with respect to
                      its first argument (Theory, the three-body integrals).
* ``explicit``     -- tier A: the grid intermediate V (eq. Ldecomp), the
                      explicit six-index L on the grid, its literal triple-grid
                      definition, the spin-orbital L, the normal-ordered
                      corrections eq. dU / eq. tcmf:1el / the zero-body
                      expectation value, and a brute-force check of the normal
                      ordering in determinant space.
* ``factorised``   -- tier B: the closed-shell working equations (Appendix B,
                      eq. tcmf:2el with the intermediates eq. tcmf:inter), for
                      any orbital subset and any diagonal per-spin density
                      (occupation numbers); the restricted open-shell
                      equations (Appendix A); the frozen-core folding of the
                      results (xTC-FC).
* ``tc2``          -- the two-body TC integrals on the grid (Theory, the
                      definition of K), as the definition written out and in
                      factorised form.
* ``gradient``     -- the differentiation loss and its exact gradient with
                      respect to the Jastrow coefficients.
* ``lowdin``       -- symmetric orthonormalisation under the grid weights.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path
and never takes an input computed by it.
"""
from . import jastrow, explicit, factorised, gradient, lowdin, tc2  # noqa: F401
