"""JAG filtered vector search for AMD Instinct MI355X (gfx950).

The library itself is ``libjag.so`` (C ABI in ``include/jag.h``); ``jag``
is its Python binding.  Importing the package does not load the library;
the first call into ``jag`` does, and fails loudly if it has not been built.
"""
__all__ = ["jag"]
