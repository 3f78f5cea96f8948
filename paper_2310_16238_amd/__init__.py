"""MI355X (gfx950) stratified Cox hot path: HIP kernels behind a C ABI (include/coxmi.h).

Submodules: ``coxmi`` (ctypes binding of libcoxmi.so), ``synth`` (seeded
synthetic inputs), ``build`` (in-tree hipcc build of the library).
"""
