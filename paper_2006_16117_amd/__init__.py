"""SIM-M indicator evaluation on MI355X (gfx950): HIP kernels behind a C ABI.

`paper_2006_16117_amd.simm` is the ctypes binding of libsimm.so (include/simm.h);
`paper_2006_16117_amd.build` compiles the library in-tree with hipcc.
"""
