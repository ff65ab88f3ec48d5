"""MI355X (gfx950) engine for expectation values of variational quantum circuits.

The computation lives in ``libqsim.so`` (HIP kernels and a C++ host planner,
C-ABI in ``include/qsim.h``); ``qsim`` is its ctypes binding, ``autograd``
wraps the adjoint gradient as a ``torch.autograd.Function``.
"""
from . import qsim  # noqa: F401  (raises ImportError when libqsim.so is not built)
from .qsim import (C64, C128, MODE_AUTO, MODE_DENSE, MODE_LIGHTCONE, MODE_LIGHTCONE_FACTORED, Context, QsimError, State,  # noqa: F401
                   lightcone_sets, plan_dense)

__all__ = ["qsim", "Context", "State", "QsimError", "lightcone_sets", "plan_dense", "C64", "C128", "MODE_AUTO",
           "MODE_DENSE", "MODE_LIGHTCONE", "MODE_LIGHTCONE_FACTORED"]
