"""FP64 CPU oracle of the coupled PMUT / DG-SEM acoustic time step.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg.  The product package never imports it.
"""
