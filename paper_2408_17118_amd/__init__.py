"""MI355X (gfx950) hot path of matrix-form ordering ICA (arXiv 2408.17118).

liboica.so holds the HIP kernels and the C ABI (include/oica.h);
``paper_2408_17118_amd.oica`` is its ctypes binding (imports torch);
``paper_2408_17118_amd.synth`` draws the seeded synthetic workloads.
"""
