"""MI355X-native local ensemble transform Kalman filter (LETKF) frame for
adaptive optics (Gray et al., arXiv:1408.7069).

The compute path is the HIP library `libletkf.so` (built for gfx950 from
`csrc/`), reached through the C ABI declared in `include/letkf.h`; `binding`
is its thin ctypes wrapper.  `workload` only makes seeded synthetic inputs.
The binding is imported lazily so that the input generators stay usable on
machines without the library; every compute call fails loudly when the
library is missing.
"""

__all__ = ["binding", "workload"]


def __getattr__(name):
    if name == "binding":
        from . import binding
        return binding
    raise AttributeError(name)
