"""MI355X-native split-form DGSEM Navier-Stokes operator (HIP, gfx950).

The operator runs in hand-written HIP kernels behind the C ABI declared in
``include/dgsem.h`` (library ``paper_2606_18927_amd/libdgsem.so``); this package
holds the thin ctypes binding (``dgsem``), the torch autograd wrapper of the RK
rollout (``autograd``) and the seeded synthetic workloads (``workloads``).
Importing the package does not load the library; the first call does, and
raises if the library is missing.
"""

__all__ = ["dgsem", "workloads"]
