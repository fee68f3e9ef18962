"""MI355X-native DD-alpha-AMG for twisted-mass Wilson-clover fermions.

The compute path is the C-ABI library ``libddamg.so`` (hand-written HIP
kernels for gfx950) reached through :mod:`paper_1611_01034_amd.ddamg`.
:mod:`paper_1611_01034_amd.synth` holds the seeded input generators.
"""
