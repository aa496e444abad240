"""MI355X (gfx950) sliding-window GDG decoder for QLDPC codes under
circuit-level noise (arXiv 2403.18901): HIP kernels behind a C ABI
(include/gdg.h) with a thin Python binding in `gdg`."""
