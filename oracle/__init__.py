"""FP64 CPU oracle of the particle-deposition step — TEST INFRASTRUCTURE ONLY.

This package is the slow, plain reference that the HIP path is checked
against.  Only the test suite, the smoke check and the benchmark's CPU
baseline leg may import it; the library and its Python binding never do, and
the oracle imports nothing from them (it shares no code, headers, constants
or helpers with the HIP path).  Its only shared dependency is the seeded
input generator package ``synthetic``, which holds none of the method.

Layout:

* ``physics``   force laws and derived constants (drag, Coulomb, van der
                Waals, soft-sphere contact, wall terms, rebound law);
* ``gather``    trilinear interpolation of the carrier field;
* ``sim``       the time step (kick-drift-kick with exponential drag), the
                wall test and the deposition tally;
* ``mfmc``      multi-fidelity Monte Carlo allocation and estimators,
                Sobol' indices (Section 3).

Everything is float64 NumPy.  Parity status of each function is stated in
its docstring; the whole coupled trajectory is "parity unpinned" beyond the
component pins (it has no closed form), see ``sim``.
"""
