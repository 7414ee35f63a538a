"""FP64 CPU oracle for matrix-form ordering ICA -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct statement of what the GPU
path computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
HIP library under ``paper_2408_17118_amd/`` and imports nothing from it; the
product path never calls it.

Modules
-------
ica   whitening, the batched kurtosis fixed point (matrix form and the
      per-candidate form), kurtosis, the ordering criterion, sign-invariant
      clustering and the Gaussianity test.
mlp   FP64 forward/backward/Adam of the small pruning network (parity
      reference for the GPU training kernels).

Parity status of each function is stated in its docstring; every function is
pinned by a ``-m "not gpu"`` test except where a docstring says
"parity unpinned".
"""
from . import ica  # noqa: F401
