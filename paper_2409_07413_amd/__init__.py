"""MI355X-native hot path of Memetic Phase Retrieval (SPRING, arXiv 2409.07413).

The computation lives in the HIP library libspr.so (C ABI in include/spr.h);
``binding`` marshals arguments to it, ``synth`` generates seeded synthetic
XFEL-shaped inputs, ``build`` compiles the library in-tree.
"""

__all__ = ["binding", "synth", "build"]
