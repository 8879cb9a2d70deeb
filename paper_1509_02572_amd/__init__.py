"""MI355X-native cut-cell finite-volume stage (Yamazaki, Satomura & Nikiforakis).

The HIP library (``csrc/``, C-ABI declared in ``include/cutcell.h``) holds the hot path.  Import
``paper_1509_02572_amd.cutcell`` for the binding; this package import itself loads nothing.
"""
__all__ = ["workloads", "cutcell"]
