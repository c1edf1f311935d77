"""MI355X-native truncated Lennard-Jones MD hot path.

Submodules:
  * ``ljmd``      -- ctypes binding of the HIP/gfx950 C-ABI library ``libljmd.so``
  * ``workloads`` -- seeded synthetic inputs (no method arithmetic)

The binding is imported lazily so that the input generators can be used
without loading the GPU library.
"""
__all__ = ["ljmd", "workloads"]


def __getattr__(name):
    if name == "ljmd":
        from . import ljmd
        return ljmd
    if name == "workloads":
        from . import workloads
        return workloads
    raise AttributeError(name)
