"""Binocular 2D Gaussian Splatting frame path for AMD Instinct MI355X.

The HIP library (libbgs.so, built by ``python -m paper_2609_30741_amd.build``)
does the work; ``api`` marshals torch tensors into its C ABI and ``synth``
generates seeded synthetic scenes and cameras.
"""
