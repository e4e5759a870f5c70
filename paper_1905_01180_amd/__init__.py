"""sb2: second-Born self-energy and GKBA collision integral on MI355X (gfx950).

The compute path is the HIP library libsb2.so (C ABI in include/sb2.h); this
package holds its build script, a ctypes binding (_lib), the autograd wrapper
(autograd) and the seeded synthetic input generators (inputs).  Importing the
package does not load the library; the first call does, and fails loudly if
it is not built.
"""
__all__ = ["inputs", "build", "ops"]
