"""MI355X-native Adaptive IDW (arXiv 1511.02186): the two-pass AIDW hot path as
hand-written gfx950 HIP kernels behind a C-ABI library (``libaidw.so``).

``paper_1511_02186_amd.aidw`` is the thin ctypes binding over that library;
``paper_1511_02186_amd.workloads`` holds the seeded input generators.  The
binding is imported lazily so that the generators load on machines without a
GPU.
"""
__all__ = ["aidw", "workloads"]


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
