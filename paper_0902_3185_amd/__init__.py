"""MI355X-native DMRG superblock H*psi (gfx950 HIP kernels behind a C ABI).

The compute lives in libdmrg.so (built from csrc/ by ``build.py``); this
package is its Python binding:

* ``superblock``  Context, Superblock (build, hpsi, adjoint, lanczos,
                  rho_truncate) -- ctypes marshalling only
* ``autograd``    hpsi as a torch.autograd.Function
* ``driver``      whole-run DMRG (infinite + finite sweeps) on top of the
                  library
"""
from ._lib import DmrgError, lib  # noqa: F401


def __getattr__(name):
    if name in ("Context", "Superblock", "build_superblock"):
        from . import superblock
        return getattr(superblock, name)
    raise AttributeError(name)
