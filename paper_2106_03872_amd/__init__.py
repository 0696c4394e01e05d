"""MI355X-native Kohn-Sham hot path: Hamiltonian application, Taylor-4
propagation and density for plane-wave real-time TDDFT (arXiv:2106.03872).

Importing the package loads nothing native; ``paper_2106_03872_amd.ks``
loads the HIP library ``libks.so`` and fails loudly when it is missing.
"""
__all__ = ["synth"]
