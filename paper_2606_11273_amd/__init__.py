"""MI355X (gfx950) implementation of the peanut-compressed two-body MFS for 2D Stokes
flow around nearly touching disks (arXiv 2606.11273).

The method runs in the HIP library ``libmfs_hip.so`` (sources in ``csrc/``, C ABI
in ``include/mfs.h``); ``native`` is its ctypes binding, ``dynamics`` a forward-Euler
driver over it and ``build`` compiles the library.  Nothing is imported eagerly:
``import paper_2606_11273_amd.native`` loads torch and the library, and fails if the
library has not been built.
"""

__all__ = ["native", "dynamics", "build"]
