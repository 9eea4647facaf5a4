"""FP64 CPU oracle of the phase-field lattice Boltzmann step (test infrastructure only).

Nothing in the product package imports this; only the tests, the smoke check and the
benchmark's CPU-baseline leg do.
"""
