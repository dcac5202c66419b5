"""MI355X (gfx950) race checker after HiRace: per-location shadow state
machines advanced by compare-and-swap in hand-written HIP kernels, behind the
C ABI declared in include/hr.h.  The ctypes binding is ``hr``."""
