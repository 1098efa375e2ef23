"""MI355X-native parallel partition refinement for DFA minimisation,
equivalence and inclusion checking.

The compute path is the C-ABI library ``libdfamin.so`` (hand-written HIP for
gfx950, built from ``csrc/``); ``binding`` marshals arguments into it.
``workloads`` holds the seeded synthetic input generators.
"""
__version__ = "0.1.0"
