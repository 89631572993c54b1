"""qsv: a dense quantum state-vector engine for AMD MI355X (gfx950).

The engine is the C-ABI library ``libqsv.so`` (hand-written HIP kernels,
declared in ``include/qsv.h``); ``paper_2502_11385_amd.qsv`` is its thin
ctypes binding.  Importing the binding requires the built library.
"""
__all__ = ["qsv"]
