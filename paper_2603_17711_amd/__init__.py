"""MI355X-native TTN-HEOM propagation (hot path of the TENSO method, arXiv 2603.17711).

The compute path is the HIP library ``libtenso.so`` (C ABI in include/tenso.h);
this package only builds its inputs (bath features, SOP term tables, trees)
and marshals arguments.  Importing the package does not load the library; the
first call that needs it does, and fails loudly if it is missing.
"""
