"""MI355X-native per-event pixel clustering behind a non-blocking acquire/produce
boundary (the offload pattern of arXiv:2004.04334, Sec. 2 and 4).

``paper_2004_04334_amd.pxcl`` is the Python binding of the HIP library
``libpxcl.so`` (C ABI: ``include/pxcl.h``); ``synth`` draws seeded synthetic events.
The binding is imported lazily so that the generators work on machines without the
built library; using the binding without the library raises.
"""

__all__ = ["pxcl", "synth", "build"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
