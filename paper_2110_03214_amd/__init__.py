"""MI355X-native MAPA allocation hot path.

The compute runs in the HIP library ``libmapa.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/mapa.h``; ``binding`` is a thin ctypes layer over
it.  ``synth`` generates seeded synthetic workloads.  Nothing is imported
eagerly, so importing the package does not load the GPU library.
"""
__all__ = ["binding", "synth"]
