"""MI355X (gfx950) hot path of the explicit relativistic PIC cycle of Melzani et
al., "Apar-T" (arXiv:1308.5892): C ABI in include/pic.h, HIP kernels in csrc/,
ctypes binding in pic.py."""
