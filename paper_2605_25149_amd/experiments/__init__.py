"""Experiment drivers built on the HIP library (finite-difference analogues of the paper's
numerical experiments)."""
