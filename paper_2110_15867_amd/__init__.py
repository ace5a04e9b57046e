"""libvlasov: split SL-MPP5 advection of f(x,u) on a 6D phase-space grid, MI355X.

The compute path is the HIP library ``libvlasov.so`` built from ``csrc/``;
``paper_2110_15867_amd.vlasov`` is its thin ctypes binding (same names as the
C entry points).  ``inputs`` builds seeded synthetic grids and fields and holds
none of the method's arithmetic.  The binding is imported lazily so that the
input generators can be used without a GPU or a built library.
"""

__all__ = ["inputs", "vlasov"]


def __getattr__(name):
    import importlib
    import importlib.util

    # submodules (vlasov, inputs, autograd, build) import on first use; only
    # other names are looked up in the binding, so building the library does
    # not need a built library
    if importlib.util.find_spec(f"{__name__}.{name}") is not None:
        return importlib.import_module(f"{__name__}.{name}")
    mod = importlib.import_module(f"{__name__}.vlasov")
    if hasattr(mod, name):
        return getattr(mod, name)
    raise AttributeError(name)
