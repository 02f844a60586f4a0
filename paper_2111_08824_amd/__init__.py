"""Learned indexed nested loop join (two-level linear RMI probe) for MI355X.

The probe runs in the HIP kernels of ``liblj.so`` behind the C ABI declared in
``include/lj.h``; ``lj`` is its Python binding.
"""
from . import lj  # noqa: F401
