"""Independent CPU oracle for the quantum-master-equation time-stepping scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP library.

Everything is plain NumPy / SciPy in complex128 / float64, written to be read
against the paper (Li, Miao, Ozhigov, "Supercomputer model of
finite-dimensional quantum electrodynamics applications"):

* ``model``        basis, Hamiltonian, decoherence operators (Sec. II
                   points 1-2; Eqs. 2-3, 8b, 10-12)
* ``evolve``       propagator, one time step, observables (Sec. II point 3;
                   the "Taylor approximation" and "unitary evolution" stages
                   of Sec. IV.B / Table III)
* ``gradients``    tangent-linear (forward-mode) derivatives of final
                   observables with respect to g, mu and gamma, and central
                   finite differences
* ``selection``    the state-space selection loop of Sec. III.B (growth
                   speed, deletion below epsilon, renormalisation, solving
                   on the kept states)
* ``closed_forms`` analytic solutions that pin the above (Rabi oscillation,
                   damped Jaynes-Cummings, photon leakage, dephasing, the
                   open-boundary lattice in its sine-mode eigenbasis)

Parity status: every function here is pinned by a test in
``tests/test_oracle_pins.py`` except where its docstring says
"parity unpinned".
"""
