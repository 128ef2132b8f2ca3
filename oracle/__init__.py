"""Plain CPU oracle for the hyperbolic-cross Hermite Galerkin method (Brumm, arXiv 1403.3511).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or link
anything under this directory; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP path.

Everything here is written for obviousness, not speed: plain NumPy in float64 /
complex128, each function citing the passage of the paper it restates.

Modules
  index      -- the index set K = {k : prod(1+k_l) <= B}, lex order, k +- e_l tables
                (Sec. 1.2, definition of the hyperbolically reduced set).
  operators  -- the coordinate operators X^(l) (Sec. 3.1, eq. DirectOperationWithX),
                formal insertion W^pol(X_K) v (Sec. 3.2, eq. Horner; Fig. 3),
                the exact Galerkin matrix on tiny sets (Sec. 1.2 + Sec. 1.1),
                product Gauss-Hermite assembly (Sec. 4.1) and the error
                split E^quad / E^red (Sec. 5.1).
  propagate  -- exponential midpoint Magnus + m-step Lanczos (Sec. 2, Fig. 4).
  surrogate  -- Gauss-Hermite projection of a smooth potential onto Hermite
                polynomials (Sec. 4.1 quadrature) and a float64 MLP with manual
                backward and Adam (test oracle for the learned coefficient path).

Pins: every function is checked by ``tests/test_oracle_*.py`` against facts the paper
or mathematics fixes (closed forms, Lemma 1, the printed error table of Fig. 9,
brute force on tiny inputs, finite differences).  Functions without such a pin say
"parity unpinned" in their docstring.
"""
