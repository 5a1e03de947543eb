"""MI355X-native alchemical short-range nonbonded kernel (lambda-dynamics hot path).

Importing the package is cheap: the HIP library is only loaded when
``paper_2608_12691_amd.alchnb`` is imported.
"""
__all__ = ["systems"]
