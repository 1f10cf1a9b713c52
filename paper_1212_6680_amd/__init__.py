"""MI355X (gfx950) SMG-preconditioned Krylov solvers behind a C ABI (include/smg.h).

Import ``paper_1212_6680_amd.smg`` for the binding; ``paper_1212_6680_amd.build``
compiles ``libsmg.so`` in-tree.
"""
