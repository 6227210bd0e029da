"""MI355X (gfx950) generic worst-case optimal join with aggregation over
dictionary-encoded uint32 tries.

The compute path is the HIP library ``liblh.so`` behind the C ABI in
``include/lh.h``; ``paper_1708_07859_amd.lh`` is its ctypes binding
(``from paper_1708_07859_amd import lh``).  Importing the package itself
loads nothing, so ``paper_1708_07859_amd.build`` runs before a build exists.
"""
