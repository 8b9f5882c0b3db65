"""MI355X (gfx950) parallel-in-time BDF-k / CQ-BDF-k solver: one
waveform-relaxation sweep solved by diagonalization in time, as hand-written
HIP kernels behind the C ABI of ``include/pint.h``.

Submodules (imported on demand so that importing the package needs neither
a GPU nor the built library):
    build     compiles ``libpint.so`` for gfx950 with hipcc
    binding   ctypes binding with the C entry-point names and a ``Plan`` wrapper
    workloads seeded synthetic inputs
"""
