"""MI355X-native DLPNO doubles-residual engine (C ABI in libdlpno.so).

The Python layer only marshals arguments: every step of the residual,
update, DIIS and adjoint runs in the HIP library.  Importing the binding
fails loudly when the library is not built.
"""
from .lib import Plan, PnoPlan, DlpnoError, library_path, FP64, FP32, BF16X2, FP16X2  # noqa: F401
