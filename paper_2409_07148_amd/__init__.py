"""MI355X (gfx950) Jump Restore chain engine.

``paper_2409_07148_amd.restore`` is the ctypes binding of the C ABI in
``include/restore.h`` (librestore.so, hand-written HIP kernels);
``paper_2409_07148_amd.build`` compiles that library in-tree with hipcc.
Importing this package loads neither, so the build step can run first.
"""
