"""MI355X-native preconditioned discrete dipole approximation (DDA) solver.

The compute path is the HIP library ``lib/libdda.so`` (C-ABI in ``include/dda.h``);
``dda`` is its ctypes binding and ``autograd`` the torch.autograd.Function for
dC_ext / d eps.  Nothing here computes on the CPU.
"""

from .dda import DDAError, Problem, load  # noqa: F401
