"""MI355X-native hot path of the Multiscale Perturbation Method for two-phase flow (MPM-2P on MRCM).

Importing the package is cheap: the HIP library is loaded by :mod:`paper_2103_11050_amd.binding`
on first use, and that module raises if the compiled library is missing.
"""

__all__ = ["inputs", "binding"]
