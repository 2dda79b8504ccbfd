"""Robust-l0 decoding of expander sketches on AMD Instinct MI355X (gfx950).

The decoder, the sketch and every kernel live in the HIP library librl0.so
(include/rl0.h); ``paper_1704_09012_amd.rl0`` is its ctypes binding.  Importing the
package loads nothing; ``instances`` draws seeded synthetic problems.
"""
__all__ = ["rl0", "instances", "build"]
