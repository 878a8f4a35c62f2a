"""MI355X-native exact temporal-motif co-mining (MG-Tree), HIP for gfx950.

The package is thin: ``api`` binds the C ABI of ``libmayura.so`` (built by
``build``), ``workloads`` draws seeded synthetic inputs.  Importing the package
loads nothing; the first API call loads the library and fails loudly if it is
missing.
"""
__all__ = ["api", "workloads", "build"]
