"""MI355X-native FFBS worldline sampler for the Hubbard model (gfx950 HIP behind a C ABI).

`fhmc` is the ctypes binding of include/fh.h; `sampler` holds the torch-facing helpers
(buffer allocation, the Sampler object and the LogZPath autograd function).
"""
