"""MI355X-native local ensemble transform Kalman filter (LETKF) frame for
adaptive optics (Gray et al., arXiv:1408.7069).

The compute path is the HIP library `libletkf.so` (built for gfx950 from
`csrc/`), reached through the C ABI declared in `include/letkf.h`;
`paper_1408_7069_amd.binding` is its thin ctypes wrapper and raises on import
when the library is missing (there is no CPU fallback).
`paper_1408_7069_amd.workload` only makes seeded synthetic inputs.
"""
