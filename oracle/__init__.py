"""FP64 CPU oracle for the randomized Chebyshev Fermi-operator expansion.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and this
package imports nothing from the product path.  The two share only the seeded
input generators in ``workloads``.

Three layers, each pinned separately by the CPU tests:

  exact      the plain definitions of F, N, E, P, Q by dense diagonalization
             (Methods: free-energy function, free energy, density matrix,
             observables);
  trunc      the same quantities with the Fermi functions replaced by their
             truncated Chebyshev series (Polynomial approximation);
  estimator  the plain randomized estimator, step by step: spectral map,
             three-term Chebyshev recurrence applied to probe vectors, moments,
             traces, the random density estimator (Random approximation) and
             the polynomial free-energy derivative (Analytical free-energy
             derivatives), with every Chebyshev vector stored (no
             checkpointing).

  overlap    the nonorthogonal-basis recurrence (H_hat S^{-1}) with exact sparse
             solves, P and Q blocks, and generalized-eigenvalue observables;
  rational   the rational (pole) expansion: a contour-integral pole fit of f and
             g, the shifted solves (H - z_k S) g_k = y by sparse LU, N, E, F,
             the P (and with an overlap Q) blocks, and the rational free-energy
             derivative (S = I).

Also: the closed-form band of the periodic simple-cubic model and the
Hellmann-Feynman force contraction (Observable response).

Parity status: every function here is pinned by a CPU test against a closed
form, a special case, brute force or a printed number of the paper; none is
"parity unpinned".
"""
