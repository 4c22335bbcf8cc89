"""MI355X-native kernelised periodogram (CS-QMI / CKP) period search.

The compute path is the HIP library ``libqmi.so`` behind the C ABI declared in ``include/qmi.h``;
``paper_1412_1840_amd.qmi`` is its thin Python binding.  Importing this package does not load the
library; the binding raises if it is missing.
"""
__all__ = ["qmi", "synth"]
