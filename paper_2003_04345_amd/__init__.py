"""MI355X (gfx950) MB4 integrator for the periodic 2D lattice NLS.

The compute path is the HIP library ``libmb4.so`` (built from ``csrc/`` by
``paper_2003_04345_amd._build``) behind the C ABI of ``include/mb4.h``;
``paper_2003_04345_amd.mb4`` is its ctypes binding.
"""
from .mb4 import (  # noqa: F401
    MB4_EDEVICE, MB4_EINVAL, MB4_ENOCONV, MB4_ENOMEM, MB4_OK, MB4Ensemble, MB4Server, MB4State,
    Mb4Error,
    load_library)
