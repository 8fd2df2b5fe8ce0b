"""MI355X-native step-based transport of electromagnetic showers.

The product is the HIP library ``libemstep.so`` (C ABI in ``include/emstep.h``);
``paper_2503_17608_amd.emstep`` is its thin ctypes binding.
"""
from .emstep import Session, exported_symbols  # noqa: F401
