"""MI355X-native (gfx950, HIP) finite-volume solver for the nonlinear
thermoviscous acoustic balance laws of Velasco-Segura & Rendon
(arXiv:1311.3004).

The method runs in libfvna.so (hand-written HIP kernels behind the C ABI of
include/fvna.h); ``paper_1311_3004_amd.fvna`` is its ctypes binding and
``paper_1311_3004_amd.inputs`` the seeded synthetic workloads.  Importing the
package itself loads nothing; importing ``fvna`` fails loudly when the
library is not built.
"""

__all__ = ["fvna", "inputs", "build"]
