"""MI355X-native server path of the two-server DPF-PIR of arXiv 2301.10904.

``pir``       -- binding of the C ABI in include/pir.h (libpir.so, HIP for gfx950)
``workloads`` -- seeded synthetic inputs (tables, query indices, arrivals)
``build``     -- in-tree hipcc build of libpir.so

Importing the package loads nothing; ``pir.load()`` loads the library and
raises if it has not been built.
"""
__all__ = ["pir", "workloads", "build"]
