"""FP64 reference oracle for Memetic Phase Retrieval (test infrastructure only).

This package is a plain, slow, deliberately unoptimised CPU implementation of
what the GPU hot path computes, written from the paper's equations and
algorithms (SPRING, arXiv 2409.07413).  It exists to check the HIP kernels.
Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import it; the product path never does.

It shares no code with the HIP library: the two meet only through the seeded
input generators (``paper_2409_07413_amd.synth``), which contain none of the
method's arithmetic.

Modules
-------
``philox``  Philox4x32-10 counter-based generator (Salmon et al., SC'11) and the
            draw conventions shared, by specification only, with the GPU.
``mpr``     Operators (FFT, projectors, ER/HIO/RAAR, shrink-wrap, fitness),
            memetic operators (RandomChoice, Reshift, CrossoverMap, mix,
            Select) and the two drivers (plain multi-start and MPR).

Parity status: every function in ``mpr`` and ``philox`` is pinned by a
``-m "not gpu"`` test against something other than itself (brute force,
closed forms, invariants, published known-answer vectors).
"""

from . import philox, mpr  # noqa: F401
