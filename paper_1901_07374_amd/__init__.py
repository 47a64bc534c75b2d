"""MI355X-native Total-Lagrangian SPH step with ductile damage.

Importing the package loads nothing native: the HIP library is opened on
first use by :mod:`paper_1901_07374_amd.tlsph`.
"""
__all__ = ["inputs", "tlsph"]
