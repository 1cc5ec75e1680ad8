"""MI355X (gfx950) implementation of the energy-conserving PIC step of the
reduced 1D and 2D relativistic Vlasov-Maxwell models (Li, arXiv 2203.06513).

The computation lives in the HIP library ``libecpic.so`` (C-ABI in
``include/ecpic.h`` and ``include/ecpic2d.h``); this package only builds and
binds it.
"""
from ._lib import (Context, EcpicError, EXPORTS, FP32_MIXED, FP64, MAP_JACOBI, MAP_SEIDEL,  # noqa: F401
                   WS_EXPLICIT, WS_MLP, WS_PREVIOUS, LIE_TROTTER, SYMMETRIC, LIB_PATH, load,
                   OK, EINVAL, ENOMEM, ENOTCONV, EDEVICE, ENONFINITE, ECFL, ESTATE)
from ._lib2d import Context2D, EXPORTS_2D  # noqa: F401,E402
