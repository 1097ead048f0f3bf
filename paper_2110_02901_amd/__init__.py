"""MI355X-native randomized mini-batch Bellman operator (arXiv 2110.02901).

The compute path is the HIP library ``libmbdp.so`` built from ``csrc/``;
``binding`` exposes its C-ABI to Python.  ``inputs`` draws seeded synthetic
MDPs.  Importing the package loads nothing; the library is loaded on first
use and a missing library raises an error.
"""
